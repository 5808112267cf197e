"""GPU edge cases of fm_apply: empty column blocks for every operator kind
(the call succeeds and writes nothing), and the largest lengths the library
accepts, 2^20, checked on outputs the oracle computes one by one from the
definitions (Fourier rows of eq. (1), circulant rows of eq. (5), Toeplitz rows
T[i, j] = t_(i - j)), forward and adjoint. The full outputs are also checked
against the FP64 FFT oracle."""

import numpy as np
import pytest

from oracle import dense, structured
from tests.gpu_util import TOL, crandn, rel_err, to_dev, to_host

pytestmark = pytest.mark.gpu


def kinds(gpu, rng):
    c = crandn(rng, 64)
    col, row = crandn(rng, 50), crandn(rng, 70)
    g = crandn(rng, (8, 6))
    rows = np.array([1, 5, 9], np.int32)
    F, C = gpu.Fourier(64), gpu.Circulant(to_dev(c))
    return {
        "fourier": F, "fourier_bluestein": gpu.Fourier(12), "circulant": C,
        "toeplitz": gpu.Toeplitz(to_dev(col), to_dev(row)), "hadamard": gpu.Hadamard(64),
        "diag": gpu.Diag(to_dev(c)), "dense": gpu.Dense(to_dev(g)),
        "select": gpu.SelectRows(64, to_dev(rows)), "product": gpu.Product(F, C),
        "sum": gpu.Sum(F, C), "kron": gpu.Kron(gpu.Fourier(8), gpu.Dense(to_dev(g))),
        "blkdiag": gpu.BlkDiag(F, C),
    }


def test_zero_columns_write_nothing(gpu):
    import torch

    from paper_1710_09578_amd import capi

    rng = np.random.default_rng(3)
    stream = torch.cuda.current_stream().cuda_stream
    for name, op in kinds(gpu, rng).items():
        m, n = op.shape
        for d, rin, rout in ((capi.FM_FWD, n, m), (capi.FM_ADJ, m, n)):
            x = to_dev(crandn(rng, (1, rin)))
            sentinel = to_dev(np.full((1, rout), 7 + 3j, np.complex64))
            y = sentinel.clone()
            capi.fm_apply(op.handle, d, 0, x, rin, y, rout, None, 0, stream)
            assert torch.equal(y, sentinel), name
        # the Python view of an empty block
        y = op.apply(to_dev(np.zeros((0, n), np.complex64)))
        assert tuple(y.shape) == (0, m), name


def _sample_rows(rng, n, k=8):
    return np.sort(np.concatenate([[0, n - 1], rng.choice(np.arange(1, n - 1), k - 2, replace=False)]))


def test_fourier_largest_length(gpu):
    n = 1 << 20
    rng = np.random.default_rng(20)
    x = crandn(rng, (1, n))
    op = gpu.Fourier(n)
    y = to_host(op @ to_dev(x))[0]
    z = to_host(op.H @ to_dev(x))[0]
    assert rel_err(y, np.fft.fft(x[0].astype(np.complex128))) <= TOL["c64"]
    ks = _sample_rows(rng, n)
    rows = dense.fourier_rows(n, ks)
    x64 = x[0].astype(np.complex128)
    assert rel_err(y[ks], rows @ x64) <= TOL["c64"]
    assert rel_err(z[ks], rows.conj() @ x64) <= TOL["c64"]  # F^H = conj(F) (F symmetric)


def test_circulant_largest_length(gpu):
    n = 1 << 20
    rng = np.random.default_rng(21)
    c, x = crandn(rng, n), crandn(rng, (1, n))
    op = gpu.Circulant(to_dev(c))
    y = to_host(op @ to_dev(x))[0]
    z = to_host(op.H @ to_dev(x))[0]
    assert rel_err(y, structured.circulant_apply_fft64(c, x)[0]) <= TOL["c64"]
    c64, x64 = c.astype(np.complex128), x[0].astype(np.complex128)
    j = np.arange(n)
    ys, zs, ry, rz = [], [], [], []
    for i in _sample_rows(rng, n):
        ry.append(np.dot(c64[(i - j) % n], x64))  # row i of C(c): c[(i - j) mod n]
        rz.append(np.dot(c64[(j - i) % n].conj(), x64))  # row i of C(c)^H
        ys.append(y[i])
        zs.append(z[i])
    assert rel_err(ys, ry) <= TOL["c64"] and rel_err(zs, rz) <= TOL["c64"]


@pytest.mark.parametrize("m,n", [(1 << 19, (1 << 19) + 1), (1 << 20, 1), (1, 1 << 20)])
def test_toeplitz_largest_embedding(gpu, m, n):
    """m + n - 1 = 2^20, the largest embedding: square-ish, one column and one
    row."""
    rng = np.random.default_rng(m + n)
    col, row = crandn(rng, m), crandn(rng, n)
    op = gpu.Toeplitz(to_dev(col), to_dev(row))
    assert op.transform_length == 1 << 20
    x, u = crandn(rng, (1, n)), crandn(rng, (1, m))
    y = to_host(op @ to_dev(x))[0]
    z = to_host(op.H @ to_dev(u))[0]
    assert rel_err(y, structured.toeplitz_apply_fft64(col, row, x)[0]) <= TOL["c64"]
    assert rel_err(z, structured.toeplitz_apply_fft64(col, row, u, True)[0]) <= TOL["c64"]
    col64, row64 = col.astype(np.complex128), row.astype(np.complex128)

    def trow(i):  # row i of T: col[i - j] for j <= i, row[j - i] above
        j = np.arange(n)
        return np.where(j <= i, col64[np.clip(i - j, 0, m - 1)], row64[np.clip(j - i, 0, n - 1)])

    def tcol(j):  # column j of T
        i = np.arange(m)
        return np.where(i >= j, col64[np.clip(i - j, 0, m - 1)], row64[np.clip(j - i, 0, n - 1)])

    ri = _sample_rows(rng, m) if m > 8 else np.arange(m)
    rj = _sample_rows(rng, n) if n > 8 else np.arange(n)
    assert rel_err(y[ri], [np.dot(trow(i), x[0]) for i in ri]) <= TOL["c64"]
    assert rel_err(z[rj], [np.dot(tcol(j).conj(), u[0]) for j in rj]) <= TOL["c64"]


def test_larger_than_largest_is_refused(gpu):
    import paper_1710_09578_amd as fm

    rng = np.random.default_rng(5)
    with pytest.raises(fm.FmError) as e:
        gpu.Toeplitz(to_dev(crandn(rng, 1 << 19)), to_dev(crandn(rng, (1 << 19) + 2)))
    assert e.value.code == "FM_E_UNSUPPORTED"
    with pytest.raises(fm.FmError) as e:
        gpu.Fourier((1 << 20) + 1)
    assert e.value.code == "FM_E_UNSUPPORTED"
