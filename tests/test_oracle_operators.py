"""Pins for the dense operator oracle.

Each check ties an oracle function to something other than itself: a
hand-derived golden fixture, an independent library routine (numpy.fft,
scipy.linalg), a closed form or an algebraic invariant. Plausible mistakes
(a transposed circulant, a sign flip in the DFT exponent, a swapped Kronecker
order, an off-by-one Toeplitz diagonal) each fail at least one of them.
"""

import numpy as np
import pytest
import scipy.linalg

from oracle import dense, structured
from tests.conftest import golden_rows

RNG = np.random.default_rng(1234)


def crand(*shape):
    return RNG.standard_normal(shape) + 1j * RNG.standard_normal(shape)


def load_complex_matrix(name):
    rows = golden_rows(name)
    return np.array([[complex(*map(float, e.split(","))) for e in r] for r in rows])


def load_real_matrix(name):
    return np.array([[float(v) for v in r] for r in golden_rows(name)])


# ---------------------------------------------------------------- Fourier
def test_fourier_golden_dft4():
    assert np.allclose(dense.fourier(4), load_complex_matrix("dft4.txt"), atol=1e-15)


@pytest.mark.parametrize("n", [1, 2, 3, 8, 12, 64])
def test_fourier_matches_numpy_fft(n):
    x = crand(5, n)
    assert np.allclose(dense.apply(dense.fourier(n), x), np.fft.fft(x, axis=1), atol=1e-12 * n)


@pytest.mark.parametrize("n", [4, 16, 60])
def test_fourier_unitary_up_to_n(n):
    f = dense.fourier(n)
    assert np.allclose(f.conj().T @ f, n * np.eye(n), atol=1e-11 * n)


def test_fourier_impulse_and_tone():
    n = 32
    f = dense.fourier(n)
    e0 = np.zeros(n); e0[0] = 1
    assert np.allclose(f @ e0, np.ones(n))
    k0 = 5
    tone = np.exp(2j * np.pi * k0 * np.arange(n) / n)
    y = f @ tone
    expect = np.zeros(n, complex); expect[k0] = n
    assert np.allclose(y, expect, atol=1e-11)


# ---------------------------------------------------------------- Circulant
def test_circulant_golden():
    assert np.array_equal(dense.circulant([1, 2, 3]).real, load_real_matrix("circulant3.txt"))


@pytest.mark.parametrize("n", [1, 5, 16, 33])
def test_dft_diagonalises_circulant(n):
    c = crand(n)
    f = dense.fourier(n)
    d = f @ dense.circulant(c) @ np.linalg.inv(f)
    assert np.allclose(d, np.diag(np.fft.fft(c)), atol=1e-10 * max(n, 1))


def test_circulant_special_cases():
    n = 7
    delta = np.zeros(n); delta[0] = 1
    assert np.allclose(dense.circulant(delta), np.eye(n))
    e1 = np.zeros(n); e1[1] = 1
    x = crand(n)
    assert np.allclose(dense.circulant(e1) @ x, np.roll(x, 1))


def test_circulant_matches_scipy():
    c = crand(9)
    assert np.allclose(dense.circulant(c), scipy.linalg.circulant(c))


# ---------------------------------------------------------------- Toeplitz
def test_toeplitz_golden():
    t = dense.toeplitz([1, 2, 3], [9, 4, 5, 6]).real
    assert np.array_equal(t, load_real_matrix("toeplitz3x4.txt"))


@pytest.mark.parametrize("m,n", [(1, 1), (1, 5), (6, 1), (7, 7), (5, 11), (13, 4)])
def test_toeplitz_matches_scipy(m, n):
    col, row = crand(m), crand(n)
    ref = scipy.linalg.toeplitz(col, np.concatenate([[col[0]], row[1:]]))
    assert np.allclose(dense.toeplitz(col, row), ref)


@pytest.mark.parametrize("m,n", [(5, 5), (3, 8), (9, 2)])
def test_toeplitz_is_block_of_circulant_embedding(m, n):
    col, row = crand(m), crand(n)
    t = dense.toeplitz(col, row)
    for L in (m + n - 1, m + n + 3, 32):
        g = np.zeros(L, complex)
        g[:m] = col
        for k in range(1, n):
            g[L - k] = row[k]
        assert np.allclose(dense.circulant(g)[:m, :n], t)


def test_circulant_is_special_toeplitz():
    c = crand(6)
    row = np.concatenate([[c[0]], c[1:][::-1]])
    assert np.allclose(dense.toeplitz(c, row), dense.circulant(c))


# ---------------------------------------------------------------- Multilevel Toeplitz
def test_ml_toeplitz_one_level_is_toeplitz():
    n = 6
    t = crand(2 * n - 1)                       # offsets -(n-1)..(n-1)
    col = t[n - 1:]                            # offsets 0..n-1
    row = t[:n][::-1]                          # offsets 0..-(n-1)
    assert np.allclose(dense.ml_toeplitz([n], t), dense.toeplitz(col, row))


def test_ml_toeplitz_separable_is_kron():
    n1, n2 = 3, 4
    t1, t2 = crand(2 * n1 - 1), crand(2 * n2 - 1)
    T1 = dense.ml_toeplitz([n1], t1)
    T2 = dense.ml_toeplitz([n2], t2)
    assert np.allclose(dense.ml_toeplitz([n1, n2], np.outer(t1, t2)), np.kron(T1, T2))


def test_ml_toeplitz_blocks_are_toeplitz():
    n1, n2 = 3, 5
    t = crand(2 * n1 - 1, 2 * n2 - 1)
    big = dense.ml_toeplitz([n1, n2], t)
    for i in range(n1):
        for j in range(n1):
            blk = big[i * n2:(i + 1) * n2, j * n2:(j + 1) * n2]
            off = t[i - j + n1 - 1]
            assert np.allclose(blk, dense.ml_toeplitz([n2], off))


# ---------------------------------------------------------------- Hadamard
def test_hadamard_golden():
    assert np.array_equal(dense.hadamard(4), load_real_matrix("hadamard4.txt").astype(int))


@pytest.mark.parametrize("n", [1, 2, 8, 64])
def test_hadamard_matches_scipy_and_is_orthogonal(n):
    h = dense.hadamard(n)
    assert np.array_equal(h, scipy.linalg.hadamard(n))
    assert np.array_equal(h @ h.T, n * np.eye(n, dtype=int))
    assert np.array_equal(h @ h, n * np.eye(n, dtype=int))


def test_hadamard_sylvester_recursion():
    h = dense.hadamard(8)
    h16 = dense.hadamard(16)
    assert np.array_equal(h16, np.block([[h, h], [h, -h]]))


def test_integer_product_wraps():
    h = dense.hadamard(4)
    x = np.array([[2**31 - 1, 2**31 - 1, 0, 0]], dtype=np.int64)
    y = dense.apply_int(h, x, 32)
    # row 0: 2*(2^31-1) = 2^32 - 2 wraps to -2 in int32
    assert y[0, 0] == -2 and y[0, 1] == 0
    assert y.dtype == np.int32


def test_kron_apply_int_matches_exact_dense():
    r = np.random.default_rng(5)
    x = r.integers(-2**31, 2**31 - 1, size=(3, 64), dtype=np.int64)
    y = structured.kron_apply_int([dense.hadamard(8), dense.hadamard(8)], x, 32)
    assert np.array_equal(y, dense.apply_int(dense.hadamard(64), x, 32))
    y64 = structured.kron_apply_int([dense.hadamard(16), dense.hadamard(4)], x, 64)
    assert np.array_equal(y64, dense.apply_int(dense.hadamard(64), x, 64))


# ---------------------------------------------------------------- Kron
def test_kron_golden():
    k = dense.kron(np.array([[1, 2], [3, 4]]), np.array([[0, 5], [6, 7]]))
    assert np.array_equal(k, load_real_matrix("kron2x2.txt").astype(int))


def test_kron_matches_numpy_and_identities():
    a, b, c = crand(2, 3), crand(4, 2), crand(3, 3)
    assert np.allclose(dense.kron(a, b, c), np.kron(np.kron(a, b), c))
    # (A (x) B)^H = A^H (x) B^H
    assert np.allclose(dense.adjoint(dense.kron(a, b)), dense.kron(a.conj().T, b.conj().T))
    # vec identity, column-major vec: (A (x) B) vec(X) = vec(B X A^T)
    x = crand(2, 3)                        # n_B x n_A
    vec = lambda m: m.reshape(-1, order="F")
    assert np.allclose(dense.kron(a, b) @ vec(x), vec(b @ x @ a.T))
    # ||A (x) B||_2 = ||A||_2 ||B||_2
    assert np.isclose(np.linalg.norm(dense.kron(a, b), 2),
                      np.linalg.norm(a, 2) * np.linalg.norm(b, 2))


def test_kron_mode_products_match_dense():
    fs = [crand(2, 3), crand(3, 2), crand(4, 4)]
    x = crand(3, 3 * 2 * 4)
    k = dense.kron(*fs)
    for adj in (False, True):
        assert np.allclose(structured.kron_apply(fs, x, adj), dense.apply(k, x, adj))


# ---------------------------------------------------------------- selection, composites
def test_select_rows():
    s = dense.select_rows(6, [0, 2, 5])
    assert np.array_equal(s @ s.conj().T, np.eye(3))
    x = crand(6)
    assert np.allclose(s @ x, x[[0, 2, 5]])
    assert np.allclose(s.conj().T @ (s @ x), np.where(np.isin(np.arange(6), [0, 2, 5]), x, 0))


def test_blkdiag_product_sum():
    a, b = crand(2, 3), crand(3, 1)
    bd = dense.blkdiag(a, b)
    assert bd.shape == (5, 4)
    assert np.allclose(bd[:2, :3], a) and np.allclose(bd[2:, 3:], b)
    assert np.allclose(bd[:2, 3:], 0) and np.allclose(bd[2:, :3], 0)
    c, d = crand(3, 4), crand(4, 2)
    assert np.allclose(dense.product(c, d), c @ d)
    assert np.allclose(dense.sum_(c, c), 2 * c)


# ---------------------------------------------------------------- every operator
OPS = {
    "fourier": lambda: dense.fourier(12),
    "diag": lambda: dense.diag(crand(7)),
    "circulant": lambda: dense.circulant(crand(10)),
    "toeplitz": lambda: dense.toeplitz(crand(6), crand(9)),
    "ml_toeplitz": lambda: dense.ml_toeplitz([2, 3], crand(3, 5)),
    "hadamard": lambda: dense.hadamard(8).astype(complex),
    "kron": lambda: dense.kron(crand(2, 3), dense.fourier(4)),
    "select": lambda: dense.select_rows(9, [1, 4, 8]),
    "product": lambda: dense.product(dense.select_rows(10, [0, 3]), dense.circulant(crand(10))),
    "blkdiag": lambda: dense.blkdiag(dense.fourier(3), dense.diag(crand(2))),
}


@pytest.mark.parametrize("name", sorted(OPS))
def test_adjoint_identity(name):
    a = OPS[name]()
    m, n = a.shape
    x, y = crand(3, n), crand(3, m)
    lhs = np.sum(np.conj(y) * dense.apply(a, x), axis=1)
    rhs = np.sum(np.conj(dense.apply(a, y, True)) * x, axis=1)
    scale = np.linalg.norm(a, 2) * np.linalg.norm(x, axis=1) * np.linalg.norm(y, axis=1)
    assert np.all(np.abs(lhs - rhs) <= 1e-13 * scale)


# ---------------------------------------------------------------- dense-free tiers
@pytest.mark.parametrize("m,n", [(7, 7), (5, 12), (30, 3), (64, 64)])
def test_toeplitz_blocks_and_fft64_match_dense(m, n):
    col, row = crand(m), crand(n)
    t = dense.toeplitz(col, row)
    for adj in (False, True):
        x = crand(3, m if adj else n)
        ref = dense.apply(t, x, adj)
        assert np.allclose(structured.toeplitz_apply_blocks(col, row, x, adj, block=4), ref)
        for L in (None, 128):
            assert np.allclose(structured.toeplitz_apply_fft64(col, row, x, adj, L=L), ref)


def test_fft64_dense_from_forward():
    """m_ij = e_i^T phi(e_j) (section "General Matrix-free Representations"):
    the FFT64 evaluation applied to unit vectors reproduces the dense matrix."""
    col, row = crand(6), crand(4)
    eye = np.eye(4)
    assert np.allclose(structured.toeplitz_apply_fft64(col, row, eye).T, dense.toeplitz(col, row))
    c = crand(8)
    assert np.allclose(structured.circulant_apply_fft64(c, np.eye(8)).T, dense.circulant(c))


def test_select_circulant_blocks_match_dense():
    c = crand(40)
    rows = np.array([0, 3, 7, 21, 39])
    a = dense.product(dense.select_rows(40, rows), dense.circulant(c))
    for adj in (False, True):
        x = crand(2, 5 if adj else 40)
        assert np.allclose(structured.select_circulant_apply(c, rows, x, adj, block=2),
                           dense.apply(a, x, adj))


def test_ml_toeplitz_fft64_matches_dense():
    nl = [3, 4]
    t = crand(5, 7)
    a = dense.ml_toeplitz(nl, t)
    for adj in (False, True):
        x = crand(2, 12)
        assert np.allclose(structured.ml_toeplitz_apply_fft64(nl, t, x, adj), dense.apply(a, x, adj))


# ---------------------------------------------------------------- block matrices
def test_blocks_single_block_and_diagonal_grid():
    a, b = crand(3, 4), crand(2, 5)
    assert np.array_equal(dense.blocks([[a]]), a)
    z1, z2 = np.zeros((3, 5)), np.zeros((2, 4))
    assert np.array_equal(dense.blocks([[a, z1], [z2, b]]), scipy.linalg.block_diag(a, b))


def test_blocks_brute_force_products():
    """y_i = sum_j A_ij x_j and x_j = sum_i A_ij^H y_i with explicit loops over
    uneven block sizes."""
    ms, ns = [3, 1, 4], [2, 5]
    grid = [[crand(m, n) for n in ns] for m in ms]
    H = dense.blocks(grid)
    x = crand(sum(ns))
    y = crand(sum(ms))
    yref = np.zeros(sum(ms), dtype=complex)
    xref = np.zeros(sum(ns), dtype=complex)
    r0 = 0
    for i, m in enumerate(ms):
        c0 = 0
        for j, n in enumerate(ns):
            for r in range(m):
                for c in range(n):
                    yref[r0 + r] += grid[i][j][r, c] * x[c0 + c]
                    xref[c0 + c] += np.conj(grid[i][j][r, c]) * y[r0 + r]
            c0 += n
        r0 += m
    assert np.allclose(H @ x, yref, atol=1e-12)
    assert np.allclose(H.conj().T @ y, xref, atol=1e-12)


def test_blocks_of_shifted_toeplitz_is_two_level_toeplitz():
    """Blocks whose generator depends on i - j only form a block-Toeplitz matrix
    with Toeplitz blocks, i.e. the 2-level Toeplitz of the combined generator."""
    n1, n2 = 3, 4
    t = crand(2 * n1 - 1, 2 * n2 - 1)
    grid = [[dense.ml_toeplitz([n2], t[i - j + n1 - 1]) for j in range(n1)] for i in range(n1)]
    assert np.array_equal(dense.blocks(grid), dense.ml_toeplitz([n1, n2], t))


def test_ml_toeplitz_rows_and_fourier_rows():
    t = crand(5, 7)
    full = dense.ml_toeplitz([3, 4], t)
    rows = [0, 5, 11, 7]
    assert np.array_equal(dense.ml_toeplitz_rows([3, 4], t, rows), full[rows])
    f = dense.fourier(12)
    assert np.allclose(dense.fourier_rows(12, [0, 3, 11]), f[[0, 3, 11]], atol=1e-14)


# ---------------------------------------------------------------- LFSR generator
def test_lfsr_golden_order4():
    ref = np.array([float(v) for v in golden_rows("lfsr4.txt")[0]])
    assert np.array_equal(dense.lfsr_sequence(4, 0b0011, 1).real, ref)


def test_lfsr_m_sequence_properties():
    """Primitive feedback polynomials give period 2^k - 1, one more -1 than +1,
    and a two-valued cyclic autocorrelation (N at lag 0, -1 elsewhere); a
    reducible one (x^4 + x^2 + 1) repeats after 6 values."""
    for order, taps in ((4, 0b0011), (5, 0b00101), (7, 0b0000011)):
        n = (1 << order) - 1
        s = dense.lfsr_sequence(order, taps, 1, 2 * n).real
        assert np.array_equal(s[:n], s[n:])
        assert not any(np.array_equal(s[:p], s[p:2 * p]) for p in range(1, n) if n % p == 0)
        assert np.sum(s[:n] < 0) == np.sum(s[:n] > 0) + 1
        ac = [np.dot(s[:n], np.roll(s[:n], -t)) for t in range(n)]
        assert ac[0] == n and all(v == -1 for v in ac[1:])
    s = dense.lfsr_sequence(4, 0b0101, 1, 12).real
    assert np.array_equal(s[:6], s[6:])
