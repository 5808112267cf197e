"""GPU parity of fm_apply (forward and adjoint) against the FP64 oracle.

Every operator is built through the C ABI from seeded inputs, applied on the
GPU, and compared column by column with the dense oracle (or, where the dense
matrix is too large, with the oracle's dense-free evaluations, which are
themselves pinned against the dense ones). Tolerance: relative L2 per column
<= 2e-5 (complex64) and <= 1e-12 (complex128); integer Hadamard and index
selection are compared bit for bit.
"""

import numpy as np
import pytest

from oracle import dense, structured
from tests.gpu_util import TOL, crandn, rel_err, to_dev, to_host

pytestmark = pytest.mark.gpu

NP = {"c64": np.complex64, "c128": np.complex128}


def torch_dt(name):
    import torch

    return {"c64": torch.complex64, "c128": torch.complex128}[name]


def check(op, a_dense, rng, prec, ncols=3, exact=False):
    m, n = a_dense.shape
    for adj in (False, True):
        x = crandn(rng, (ncols, m if adj else n), NP[prec])
        y = to_host(op.apply(to_dev(x), adjoint=adj))
        ref = dense.apply(a_dense, x, adj)
        err = rel_err(y, ref)
        assert err <= TOL[prec], f"adj={adj}: rel err {err:.3e}"


# ---------------------------------------------------------------- Fourier
@pytest.mark.parametrize("prec", ["c64", "c128"])
@pytest.mark.parametrize("n", [1, 2, 4, 8, 16, 32, 128, 512, 1024, 4096, 8192])
def test_fourier_dense(gpu, prec, n):
    rng = np.random.default_rng(n)
    op = gpu.Fourier(n, torch_dt(prec))
    if n <= 2048:
        check(op, dense.fourier(n), rng, prec, ncols=5)
    else:
        for adj in (False, True):
            x = crandn(rng, (3, n), NP[prec])
            y = to_host(op.apply(to_dev(x), adjoint=adj))
            ref = np.fft.ifft(x, axis=1) * n if adj else np.fft.fft(x, axis=1)
            assert rel_err(y, ref) <= TOL[prec]


@pytest.mark.parametrize("prec", ["c64", "c128"])
@pytest.mark.parametrize("n", [16384, 65536, 131072])
def test_fourier_four_step(gpu, prec, n):
    """Lengths above one work-group's LDS (two transform passes + transpose);
    reference: numpy.fft in complex128 (pinned to the dense DFT in the oracle
    tests)."""
    rng = np.random.default_rng(n + 1)
    op = gpu.Fourier(n, torch_dt(prec))
    for adj in (False, True):
        x = crandn(rng, (2, n), NP[prec])
        y = to_host(op.apply(to_dev(x), adjoint=adj))
        ref = np.fft.ifft(x.astype(np.complex128), axis=1) * n if adj else np.fft.fft(x.astype(np.complex128), axis=1)
        assert rel_err(y, ref) <= TOL[prec]


# ---------------------------------------------------------------- Circulant
@pytest.mark.parametrize("prec", ["c64", "c128"])
@pytest.mark.parametrize("n", [1, 2, 8, 16, 64, 256, 1024, 2048])
def test_circulant_dense(gpu, prec, n):
    rng = np.random.default_rng(100 + n)
    c = crandn(rng, n, NP[prec])
    op = gpu.Circulant(to_dev(c))
    check(op, dense.circulant(c), rng, prec, ncols=7)


def test_circulant_1024_x16_config(gpu):
    """Circulant N=1024, CN(0,1) generator (seed 0), 16 CN(0,1) columns."""
    from workloads import circulant_1024

    c, x = circulant_1024()
    op = gpu.Circulant(to_dev(c))
    a = dense.circulant(c)
    y = to_host(op @ to_dev(x))
    assert rel_err(y, dense.apply(a, x)) <= TOL["c64"]
    z = to_host(op.H @ to_dev(x))
    assert rel_err(z, dense.apply(a, x, True)) <= TOL["c64"]


@pytest.mark.parametrize("prec", ["c64", "c128"])
@pytest.mark.parametrize("n", [16, 32, 64, 128, 256, 512, 1024])
def test_few_columns_same_bits_as_many(gpu, prec, n):
    """A launch of few work-groups loads the spectrum and twiddle seeds with
    the input (latency form); a launch of many does not. Both take the same
    arithmetic: the first columns of a wide block equal the same columns
    applied alone, bit for bit, and both match the oracle."""
    rng = np.random.default_rng(900 + n)
    c = crandn(rng, n, NP[prec])
    op = gpu.Circulant(to_dev(c))
    wide = crandn(rng, (512 * (1024 // n), n), NP[prec])  # 512 one-wave work-groups of 1024 // n transforms
    few = wide[:16].copy()                                # at most 16
    a = dense.circulant(c)
    for adj in (False, True):
        yw = to_host(op.apply(to_dev(wide), adjoint=adj))
        yf = to_host(op.apply(to_dev(few), adjoint=adj))
        assert np.array_equal(yw[:16], yf), f"adj={adj}: latency form differs from the throughput form"
        assert rel_err(yf, dense.apply(a, few, adj)) <= TOL[prec]


@pytest.mark.parametrize("prec", ["c64", "c128"])
@pytest.mark.parametrize("n", [4096, 8192, 16384, 65536, 131072])
def test_circulant_large(gpu, prec, n):
    rng = np.random.default_rng(200 + n)
    c = crandn(rng, n, NP[prec])
    op = gpu.Circulant(to_dev(c))
    for adj in (False, True):
        x = crandn(rng, (3, n), NP[prec])
        y = to_host(op.apply(to_dev(x), adjoint=adj))
        ref = structured.circulant_apply_fft64(c, x, adj)
        assert rel_err(y, ref) <= TOL[prec]


# ---------------------------------------------------------------- Toeplitz
@pytest.mark.parametrize("prec", ["c64", "c128"])
@pytest.mark.parametrize("m,n", [(1, 1), (1, 7), (9, 1), (5, 5), (100, 37), (37, 100), (1000, 1000),
                                 (1500, 700), (2049, 2048)])
def test_toeplitz_dense(gpu, prec, m, n):
    rng = np.random.default_rng(m * 7 + n)
    col, row = crandn(rng, m, NP[prec]), crandn(rng, n, NP[prec])
    op = gpu.Toeplitz(to_dev(col), to_dev(row))
    check(op, dense.toeplitz(col, row), rng, prec, ncols=4)


@pytest.mark.parametrize("prec", ["c64", "c128"])
@pytest.mark.parametrize("m,n,n2", [(5000, 5000, 3), (3000, 7000, 3), (9000, 9000, 5), (11000, 11000, 6),
                                    (17000, 17000, 9), (20000, 20000, 10), (23000, 23000, 12),
                                    (27000, 27000, 16), (36000, 36000, 20), (50000, 20000, 20),
                                    (45000, 45000, 24), (55000, 55000, 30)])
def test_toeplitz_mixed_embedding(gpu, prec, m, n, n2):
    """Toeplitz operators whose embedding length is 4096 * n2 with n2 not a
    power of two (the smallest admissible length >= m + n - 1): folded rows
    (n2 <= 8), separate strided passes, two threads per column (n2 >= 20);
    forward, adjoint and the accumulate path, against the FP64 FFT oracle."""
    assert 4096 * n2 >= m + n - 1 > 4096 * max(v for v in (1, 2, 3, 4, 5, 6, 8, 9, 10, 12, 16, 20, 24)
                                                if 4096 * v < m + n - 1)
    rng = np.random.default_rng(m + 7 * n)
    col, row = crandn(rng, m, NP[prec]), crandn(rng, n, NP[prec])
    op = gpu.Toeplitz(to_dev(col), to_dev(row))
    assert op.transform_length == 4096 * n2
    for adj in (False, True):
        x = crandn(rng, (3, m if adj else n), NP[prec])
        y = to_host(op.apply(to_dev(x), adjoint=adj))
        assert rel_err(y, structured.toeplitz_apply_fft64(col, row, x, adj)) <= TOL[prec], adj
    x = crandn(rng, (2, n), NP[prec])
    y = to_host(gpu.Sum(op, op) @ to_dev(x))
    assert rel_err(y, 2 * structured.toeplitz_apply_fft64(col, row, x)) <= TOL[prec]


@pytest.mark.parametrize("kind,n,ncols", [("circulant", 16384, 64), ("circulant", 8192, 83),
                                           ("toeplitz", 5000, 83), ("toeplitz", 12000, 70)])
def test_folded_rows_wide_blocks(gpu, kind, n, ncols):
    """Folded four-step rows on 64 or more columns, where the rows of each
    column are placed on one XCD (83 columns: the last group of 8 is padded
    with work-groups that exit): forward and adjoint against the FP64 FFT
    oracle, complex64."""
    rng = np.random.default_rng(n + ncols)
    x = crandn(rng, (ncols, n))
    if kind == "circulant":
        c = crandn(rng, n)
        op = gpu.Circulant(to_dev(c))
        refs = [structured.circulant_apply_fft64(c, x, adj) for adj in (False, True)]
    else:
        col, row = crandn(rng, n), crandn(rng, n)
        op = gpu.Toeplitz(to_dev(col), to_dev(row))
        refs = [structured.toeplitz_apply_fft64(col, row, x, adj) for adj in (False, True)]
    for adj, ref in zip((False, True), refs):
        assert rel_err(to_host(op.apply(to_dev(x), adjoint=adj)), ref) <= TOL["c64"], adj


def test_transform_length(gpu):
    """The cyclic length each kind reports: n for power-of-two Fourier and
    Circulant, the embedding length for Toeplitz (power of two up to 4096,
    then the smaller of the power of two and 4096 * n2) and for the sizes
    served through one, 0 otherwise."""
    rng = np.random.default_rng(2)

    def toep(m, n):
        return gpu.Toeplitz(to_dev(crandn(rng, m, np.complex64)), to_dev(crandn(rng, n, np.complex64)))

    assert gpu.Fourier(256).transform_length == 256
    assert gpu.Circulant(to_dev(crandn(rng, 512, np.complex64))).transform_length == 512
    assert toep(100, 100).transform_length == 256
    assert toep(2049, 2048).transform_length == 4096
    assert toep(2049, 2049).transform_length == 8192  # 8192 < 3 * 4096
    assert toep(5000, 5000).transform_length == 3 * 4096
    assert toep(6145, 6145).transform_length == 16384
    assert toep(40000, 40000).transform_length == 20 * 4096
    assert toep(65536, 65536).transform_length == 131072
    assert gpu.Circulant(to_dev(crandn(rng, 1000, np.complex64))).transform_length == 2048
    assert gpu.Diag(to_dev(crandn(rng, 8, np.complex64))).transform_length == 0
    assert gpu.Fourier(12).transform_length == 32  # Bluestein: Toeplitz 12 x 12, 23 <= 32
    assert gpu.Fourier(3001).transform_length == 8192
    assert gpu.Hadamard(64).transform_length == 0


@pytest.mark.parametrize("prec", ["c64", "c128"])
@pytest.mark.parametrize("m,n", [(4097, 4097), (9000, 6000), (20000, 20000), (40000, 40000), (65536, 65536)])
def test_toeplitz_large(gpu, prec, m, n):
    rng = np.random.default_rng(m + 3 * n)
    col, row = crandn(rng, m, NP[prec]), crandn(rng, n, NP[prec])
    op = gpu.Toeplitz(to_dev(col), to_dev(row))
    for adj in (False, True):
        x = crandn(rng, (2, m if adj else n), NP[prec])
        y = to_host(op.apply(to_dev(x), adjoint=adj))
        ref = structured.toeplitz_apply_fft64(col, row, x, adj)
        assert rel_err(y, ref) <= TOL[prec]
    # sampled rows straight from the definition (no FFT in the reference)
    x = crandn(rng, (1, n), NP[prec])
    y = to_host(op @ to_dev(x))[0]
    rows = rng.choice(m, size=8, replace=False)
    for i in rows:
        trow = np.where(np.arange(n) <= i, col[np.clip(i - np.arange(n), 0, m - 1)],
                        row[np.clip(np.arange(n) - i, 0, n - 1)]).astype(np.complex128)
        ref_i = np.dot(trow, x[0].astype(np.complex128))
        assert abs(y[i] - ref_i) <= 1e-4 * np.linalg.norm(trow) * np.linalg.norm(x[0])


# ---------------------------------------------------------------- multilevel Toeplitz
@pytest.mark.parametrize("prec", ["c64", "c128"])
@pytest.mark.parametrize("levels", [[5], [3, 4], [7, 9], [2, 3, 4]])
def test_ml_toeplitz(gpu, prec, levels):
    rng = np.random.default_rng(sum(levels))
    t = crandn(rng, tuple(2 * v - 1 for v in levels), NP[prec])
    op = gpu.MLToeplitz(levels, to_dev(t))
    check(op, dense.ml_toeplitz(levels, t), rng, prec, ncols=3)


# ---------------------------------------------------------------- Hadamard
@pytest.mark.parametrize("prec", ["c64", "c128"])
@pytest.mark.parametrize("n", [1, 2, 8, 16, 32, 1024, 2048])
def test_hadamard_complex(gpu, prec, n):
    rng = np.random.default_rng(n + 5)
    op = gpu.Hadamard(n, torch_dt(prec))
    check(op, dense.hadamard(n).astype(np.complex128), rng, prec, ncols=5)


@pytest.mark.parametrize("bits", [32, 64])
@pytest.mark.parametrize("n", [1, 4, 16, 64, 512, 4096, 32768, 65536])
def test_hadamard_integer_bit_exact(gpu, bits, n):
    import torch

    from oracle import structured

    rng = np.random.default_rng(bits + n)
    npdt = np.int32 if bits == 32 else np.int64
    if n <= 512:
        info = np.iinfo(npdt)
        x = rng.integers(info.min, info.max, size=(3, n), dtype=npdt, endpoint=True)
        ref = dense.apply_int(dense.hadamard(n), x, bits)
    else:
        # int32: full range (the sums wrap); int64: |x| < 2^40 so the int64
        # reference sums stay exact
        lim = 2**31 if bits == 32 else 2**40
        x = rng.integers(-lim, lim - 1, size=(3, n), dtype=np.int64).astype(npdt)
        a = 1 << (n.bit_length() - 1) // 2
        ref = structured.kron_apply_int([dense.hadamard(n // a), dense.hadamard(a)], x, bits)
    op = gpu.Hadamard(n, torch.int32 if bits == 32 else torch.int64)
    y = to_host(op @ to_dev(x))
    assert np.array_equal(y, ref)
    # H is its own adjoint
    z = to_host(op.H @ to_dev(x))
    assert np.array_equal(z, y)


@pytest.mark.parametrize("prec", ["c64", "c128"])
def test_hadamard_two_pass(gpu, prec):
    n = 32768
    rng = np.random.default_rng(7)
    x = crandn(rng, (2, n), NP[prec])
    op = gpu.Hadamard(n, torch_dt(prec))
    y = to_host(op @ to_dev(x)).astype(np.complex128)
    # reference by the Kronecker identity H_n = H_a (x) H_b with dense factors
    ref = structured.kron_apply([dense.hadamard(256), dense.hadamard(128)], x)
    assert rel_err(y, ref) <= TOL[prec]


# ---------------------------------------------------------------- Diag, Dense, selection
@pytest.mark.parametrize("prec", ["c64", "c128"])
def test_diag_dense_select(gpu, prec):
    rng = np.random.default_rng(11)
    d = crandn(rng, 300, NP[prec])
    check(gpu.Diag(to_dev(d)), dense.diag(d), rng, prec)
    a = crandn(rng, (37, 53), NP[prec])
    check(gpu.Dense(to_dev(a)), a.astype(np.complex128), rng, prec)
    import torch

    rows = np.sort(rng.choice(500, 77, replace=False)).astype(np.int32)
    s = gpu.SelectRows(500, to_dev(rows), torch_dt(prec))
    for adj in (False, True):
        x = crandn(rng, (4, 77 if adj else 500), NP[prec])
        y = to_host(s.apply(to_dev(x), adjoint=adj))
        ref = dense.apply(dense.select_rows(500, rows), x, adj)
        assert np.array_equal(y.astype(np.complex128), ref)


@pytest.mark.parametrize("bits", [32, 64])
def test_select_integer_bit_exact(gpu, bits):
    import torch

    rng = np.random.default_rng(bits)
    npdt = np.int32 if bits == 32 else np.int64
    rows = rng.permutation(1000)[:333].astype(np.int32)  # unsorted, distinct
    s = gpu.SelectRows(1000, to_dev(rows), torch.int32 if bits == 32 else torch.int64)
    x = rng.integers(-1000, 1000, size=(2, 1000)).astype(npdt)
    assert np.array_equal(to_host(s @ to_dev(x)), x[:, rows])
    u = rng.integers(-1000, 1000, size=(2, 333)).astype(npdt)
    z = np.zeros((2, 1000), npdt)
    z[:, rows] = u
    assert np.array_equal(to_host(s.H @ to_dev(u)), z)


# ---------------------------------------------------------------- composites
@pytest.mark.parametrize("prec", ["c64", "c128"])
def test_composites(gpu, prec):
    import torch

    rng = np.random.default_rng(21)
    dt = torch_dt(prec)
    c = crandn(rng, 64, NP[prec])
    col, row = crandn(rng, 40, NP[prec]), crandn(rng, 64, NP[prec])
    d = crandn(rng, 64, NP[prec])
    g = crandn(rng, (5, 3), NP[prec])
    C = gpu.Circulant(to_dev(c))
    T = gpu.Toeplitz(to_dev(col), to_dev(row))
    D = gpu.Diag(to_dev(d))
    G = gpu.Dense(to_dev(g))
    F = gpu.Fourier(8, dt)
    H = gpu.Hadamard(4, dt)
    rows = np.array([1, 5, 9, 30, 63], np.int32)
    S = gpu.SelectRows(64, to_dev(rows), dt)
    cd, td, dd, gd = dense.circulant(c), dense.toeplitz(col, row), dense.diag(d), g.astype(np.complex128)
    fd, hd, sd = dense.fourier(8), dense.hadamard(4).astype(complex), dense.select_rows(64, rows)
    check(gpu.Product(T, C, D), td @ cd @ dd, rng, prec)
    check(S @ C, sd @ cd, rng, prec)
    check(gpu.Sum(C, D, C.H), cd + dd + cd.conj().T, rng, prec)
    check(gpu.Kron(F, G), dense.kron(fd, gd), rng, prec)
    check(gpu.Kron(G, F, H), dense.kron(gd, fd, hd), rng, prec)
    check(gpu.Kron(H, gpu.Product(G, G.H), F), dense.kron(hd, gd @ gd.conj().T, fd), rng, prec)
    check(gpu.BlkDiag(C, G, F), dense.blkdiag(cd, gd, fd), rng, prec)
    check(gpu.Kron(gpu.BlkDiag(F, H), G), dense.kron(dense.blkdiag(fd, hd), gd), rng, prec)
    check(gpu.Product(gpu.Kron(F, H), gpu.BlkDiag(gpu.Diag(to_dev(d[:8])), F, H, H, F)),
          dense.kron(fd, hd) @ dense.blkdiag(dense.diag(d[:8]), fd, hd, hd, fd), rng, prec)
    check(T.H, td.conj().T, rng, prec)
    check(gpu.Product(S, C).H, (sd @ cd).conj().T, rng, prec)


@pytest.mark.parametrize("prec", ["c64", "c128"])
@pytest.mark.parametrize("kind,m,n,nsel,ncols", [
    ("circulant", 8, 8, 3, 5),            # transforms of fewer than 16 points
    ("circulant", 1024, 1024, 100, 7),    # one-wave single pass
    ("circulant", 4096, 4096, 1000, 3),   # 4096-value single pass
    ("circulant", 16384, 16384, 2048, 5),   # folded rows
    ("circulant", 16384, 16384, 2048, 70),  # folded rows grouped per XCD
    ("circulant", 65536, 65536, 4096, 2),   # separate strided passes
    ("toeplitz", 3000, 2000, 333, 4),     # L = 8192
    ("toeplitz", 700, 1500, 700, 3),      # every output row selected
    ("toeplitz", 5000, 5000, 999, 2),     # L = 12288 = 4096 * 3: the two-step path
])
def test_selection_fused_into_convolution(gpu, prec, kind, m, n, nsel, ncols):
    """S C: the selection applied in C's last pass (forward) gives the same
    bits as the two steps S (C x); forward and adjoint match the oracle and
    accumulate in a Sum."""
    rng = np.random.default_rng(m + 3 * n + nsel + ncols)
    if kind == "circulant":
        c = crandn(rng, n, NP[prec])
        C = gpu.Circulant(to_dev(c))
        ref = lambda x, adj: structured.circulant_apply_fft64(c, x, adj)  # noqa: E731
    else:
        col, row = crandn(rng, m, NP[prec]), crandn(rng, n, NP[prec])
        C = gpu.Toeplitz(to_dev(col), to_dev(row))
        ref = lambda x, adj: structured.toeplitz_apply_fft64(col, row, x, adj)  # noqa: E731
    rows = np.sort(rng.choice(m, nsel, replace=False)).astype(np.int32)
    S = gpu.SelectRows(m, to_dev(rows), torch_dt(prec))
    A = gpu.Product(S, C)
    x = crandn(rng, (ncols, n), NP[prec])
    y = to_host(A @ to_dev(x))
    assert np.array_equal(y, to_host(S @ (C @ to_dev(x)))), "forward differs from the two steps"
    assert rel_err(y, ref(x, False)[:, rows]) <= TOL[prec]
    u = crandn(rng, (ncols, nsel), NP[prec])
    z = to_host(A.H @ to_dev(u))
    assert np.array_equal(z, to_host(C.H @ (S.H @ to_dev(u)))), "adjoint differs from the two steps"
    su = np.zeros((ncols, m), NP[prec])
    su[:, rows] = u
    assert rel_err(z, ref(su, True)) <= TOL[prec]
    y2 = to_host(gpu.Sum(A, A) @ to_dev(x))
    assert rel_err(y2, 2 * ref(x, False)[:, rows]) <= TOL[prec]
    z2 = to_host(gpu.Sum(A, A).H @ to_dev(u))
    assert rel_err(z2, 2 * ref(su, True)) <= TOL[prec]


@pytest.mark.parametrize("prec", ["c64", "c128"])
@pytest.mark.parametrize("n1,n2", [(1024, 64), (2048, 37), (4096, 5), (512, 3)])
def test_long_transforms_along_a_strided_axis(gpu, prec, n1, n2):
    """Fourier(n1) along the slow axis of Kron(F_n1, F_n2): strided transforms
    of 512..4096 points whose work-group tiles hold 8 or fewer vectors, i.e.
    row segments shorter than a 128-byte line (the tiles of a line are
    regrouped onto one XCD); ragged tile counts (37, 5, 3 vectors). Oracle:
    mode products with the dense factors."""
    import torch

    rng = np.random.default_rng([n1, n2])
    dt = torch_dt(prec)
    K = gpu.Kron(gpu.Fourier(n1, dt), gpu.Fourier(n2, dt))
    fs = [dense.fourier(n1), dense.fourier(n2)]
    for adj in (False, True):
        x = crandn(rng, (5, n1 * n2), NP[prec])
        y = to_host(K.apply(to_dev(x), adjoint=adj))
        err = rel_err(y, structured.kron_apply(fs, x, adjoint_dir=adj))
        assert err <= TOL[prec], f"adj={adj}: rel err {err:.3e}"


@pytest.mark.parametrize("prec", ["c64", "c128"])
def test_adjoint_identity(gpu, prec):
    """<A x, y> = <x, A^H y> for a composed operator, on the GPU."""
    import torch

    rng = np.random.default_rng(5)
    c = crandn(rng, 4096, NP[prec])
    rows = np.sort(rng.choice(4096, 1000, replace=False)).astype(np.int32)
    A = gpu.Product(gpu.SelectRows(4096, to_dev(rows), torch_dt(prec)), gpu.Circulant(to_dev(c)))
    x = crandn(rng, (4, 4096), NP[prec])
    y = crandn(rng, (4, 1000), NP[prec])
    ax = to_host(A @ to_dev(x)).astype(np.complex128)
    ahy = to_host(A.H @ to_dev(y)).astype(np.complex128)
    lhs = np.sum(np.conj(y.astype(np.complex128)) * ax, axis=1)
    rhs = np.sum(np.conj(ahy) * x.astype(np.complex128), axis=1)
    nrm = np.max(np.abs(np.fft.fft(c.astype(np.complex128))))
    scale = nrm * np.linalg.norm(x, axis=1) * np.linalg.norm(y, axis=1)
    tol = 1e-5 if prec == "c64" else 1e-13
    assert np.all(np.abs(lhs - rhs) <= tol * scale)


def test_leading_dimension_and_views(gpu):
    """Blocks with ld > rows (column views of a wider buffer)."""
    import torch

    rng = np.random.default_rng(3)
    c = crandn(rng, 256, np.complex64)
    op = gpu.Circulant(to_dev(c))
    big = to_dev(crandn(rng, (5, 300), np.complex64))
    x = big[:, :256]
    assert x.stride(0) == 300
    y = torch.zeros((5, 400), dtype=torch.complex64, device="cuda")
    op.apply(x, out=y[:, :256])
    ref = dense.apply(dense.circulant(c), to_host(x))
    assert rel_err(to_host(y[:, :256]), ref) <= TOL["c64"]
    assert np.all(to_host(y[:, 256:]) == 0)
    # S C with the selection inside the transform (single pass and four-step)
    for n, nsel in ((256, 40), (16384, 300)):
        c = crandn(rng, n, np.complex64)
        rows = np.sort(rng.choice(n, nsel, replace=False)).astype(np.int32)
        A = gpu.Product(gpu.SelectRows(n, to_dev(rows)), gpu.Circulant(to_dev(c)))
        big = to_dev(crandn(rng, (3, n + 17), np.complex64))
        x = big[:, :n]
        y = torch.zeros((3, nsel + 9), dtype=torch.complex64, device="cuda")
        A.apply(x, out=y[:, :nsel])
        ref = structured.circulant_apply_fft64(c, to_host(x))[:, rows]
        assert rel_err(to_host(y[:, :nsel]), ref) <= TOL["c64"]
        assert np.all(to_host(y[:, nsel:]) == 0)
        u = big[:, :nsel]
        z = torch.zeros((3, n + 5), dtype=torch.complex64, device="cuda")
        A.apply(u, adjoint=True, out=z[:, :n])
        su = np.zeros((3, n), np.complex64)
        su[:, rows] = to_host(u)
        assert rel_err(to_host(z[:, :n]), structured.circulant_apply_fft64(c, su, True)) <= TOL["c64"]
        assert np.all(to_host(z[:, n:]) == 0)


# ---------------------------------------------------------------- Kronecker workload at full size
def test_kron_hfg_full_size_sampled_columns(gpu):
    """Kron(H_1024, F_256, G_32) on 64 columns of 8,388,608 rows (complex64,
    4 GiB per block), forward and adjoint, in the launch configuration the
    benchmark times. Oracle: mode products with the dense complex128 factors on
    8 seeded columns (columns are independent, so the check is exact for them)."""
    import torch

    from workloads import kron_hfg

    g, X = kron_hfg(device=torch.device("cuda:0"))
    K = gpu.Kron(gpu.Hadamard(1024), gpu.Fourier(256), gpu.Dense(to_dev(g)))
    Y = K @ X
    Z = K.H @ X
    cols = [0, 9, 17, 28, 33, 47, 52, 63]
    xs = to_host(X[cols])
    fs = [dense.hadamard(1024), dense.fourier(256), g]
    ey = rel_err(to_host(Y[cols]), structured.kron_apply(fs, xs))
    ez = rel_err(to_host(Z[cols]), structured.kron_apply(fs, xs, adjoint_dir=True))
    print(f"kron H1024 F256 G32 full size: fwd {ey:.2e} adj {ez:.2e}")
    assert ey <= TOL["c64"] and ez <= TOL["c64"]


def test_circulant_wide_block_sampled_columns(gpu):
    """The 1024-point circulant on 65,536 CN(0,1) columns (512 MiB per block),
    forward and adjoint, in the launch configuration the benchmark times.
    Oracle: the dense complex128 circulant on 64 seeded columns."""
    import torch

    from workloads import many_columns

    c, X = many_columns(device=torch.device("cuda:0"))
    op = gpu.Circulant(to_dev(c))
    Y = op @ X
    Z = op.H @ Y
    cols = np.sort(np.random.default_rng(7).choice(X.shape[0], 64, replace=False))
    a = dense.circulant(c)
    xs = to_host(X[cols])
    ey = rel_err(to_host(Y[cols]), dense.apply(a, xs))
    ez = rel_err(to_host(Z[cols]), dense.apply(a, to_host(Y[cols]), True))
    print(f"circulant 1024 x 65536: fwd {ey:.2e} adj {ez:.2e}")
    assert ey <= TOL["c64"] and ez <= TOL["c64"]


@pytest.mark.parametrize("prec", ["c64", "c128"])
@pytest.mark.parametrize("shape", [(32, 32), (20, 12), (5, 40), (64, 64)])
@pytest.mark.parametrize("real", [True, False])
def test_dense_mode_product_many_vectors(gpu, prec, shape, real):
    """A small dense factor along the contiguous axis of many vectors (the
    register-blocked path): Kron(I_P, G) with P vectors per column, real and
    complex G, forward and adjoint, ragged vector counts."""
    import torch

    if prec == "c128" and max(shape) > 32:
        pytest.skip("complex128 register path covers factors up to 32")
    rng = np.random.default_rng(shape[0] * 100 + shape[1])
    m, n = shape
    g = crandn(rng, shape, NP[prec])
    if real:
        g = g.real.astype(NP[prec])
    P = 1300  # vectors per column: not a multiple of the 256-vector tile
    ones = to_dev(np.ones(P, NP[prec]))
    K = gpu.Kron(gpu.Diag(ones), gpu.Dense(to_dev(g)))
    for adj in (False, True):
        rin, rout = (m, n) if adj else (n, m)
        x = crandn(rng, (3, P * rin), NP[prec])
        y = to_host(K.apply(to_dev(x), adjoint=adj))
        ga = g.astype(np.complex128)
        op = ga.conj().T if adj else ga
        ref = np.einsum("rk,cpk->cpr", op, x.astype(np.complex128).reshape(3, P, rin)).reshape(3, P * rout)
        assert rel_err(y, ref) <= TOL[prec], (adj, rel_err(y, ref))
    # unpacked columns (leading dimension above the rows) through the C ABI
    from paper_1710_09578_amd import capi

    x = crandn(rng, (2, P * n + 7), NP[prec])
    y = torch.zeros((2, P * m + 5), dtype=torch_dt(prec), device="cuda")
    capi.fm_apply(K.handle, capi.FM_FWD, 2, to_dev(x), P * n + 7, y, P * m + 5, None, 0,
                  torch.cuda.current_stream().cuda_stream)
    ref = np.einsum("rk,cpk->cpr", g.astype(np.complex128),
                    x[:, :P * n].astype(np.complex128).reshape(2, P, n)).reshape(2, P * m)
    yh = to_host(y)
    assert rel_err(yh[:, :P * m], ref) <= TOL[prec] and np.all(yh[:, P * m:] == 0)


@pytest.mark.parametrize("prec", ["c64", "c128"])
@pytest.mark.parametrize("nf,gshape,real", [(16, (32, 32), True), (64, (20, 12), False), (256, (32, 32), False),
                                            (512, (5, 3), True), (128, (12, 20), True)])
def test_kron_fourier_dense_slab(gpu, prec, nf, gshape, real):
    """Kron(H_4, F_nf, G) and Kron(F_nf, G): the last two factors go through
    the fused slab pass (complex64) or the per-factor passes (complex128);
    forward, adjoint and accumulation (Sum of two Kronecker products)."""
    rng = np.random.default_rng(nf + gshape[0])
    g = crandn(rng, gshape, NP[prec])
    if real:
        g = g.real.astype(NP[prec])
    gd = g.astype(np.complex128)
    F = gpu.Fourier(nf, torch_dt(prec))
    G = gpu.Dense(to_dev(g))
    H = gpu.Hadamard(4, torch_dt(prec))
    fs_full = [dense.hadamard(4).astype(complex), dense.fourier(nf), gd]
    for op, fs in ((gpu.Kron(H, F, G), fs_full), (gpu.Kron(F, G), fs_full[1:])):
        m, n = op.shape
        for adj in (False, True):
            x = crandn(rng, (3, m if adj else n), NP[prec])
            y = to_host(op.apply(to_dev(x), adjoint=adj))
            ref = structured.kron_apply(fs, x, adjoint_dir=adj)
            assert rel_err(y, ref) <= TOL[prec], (adj, rel_err(y, ref))
    K = gpu.Kron(F, G)
    S2 = gpu.Sum(K, K)
    x = crandn(rng, (2, K.shape[1]), NP[prec])
    y = to_host(S2 @ to_dev(x))
    assert rel_err(y, 2 * structured.kron_apply(fs_full[1:], x)) <= TOL[prec]
