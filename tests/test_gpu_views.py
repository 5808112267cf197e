"""GPU parity of the views and derived operators (conj, transpose, Gramian,
structured inverse) and of the sizes served through an embedding: Fourier of
any n (Bluestein), circulants of any n, the LFSR circulant. Oracle: the dense
FP64 matrices of their definitions (conj / transpose / A^H A / numpy's
inverse of the dense matrix)."""

import numpy as np
import pytest

from oracle import dense
from tests.gpu_util import TOL, crandn, rel_err, to_dev, to_host

pytestmark = pytest.mark.gpu

NP = {"c64": np.complex64, "c128": np.complex128}


def tdt(prec):
    import torch

    return {"c64": torch.complex64, "c128": torch.complex128}[prec]


def check_both(op, a, rng, prec, ncols=3, tol=None):
    tol = TOL[prec] if tol is None else tol
    m, n = a.shape
    x = crandn(rng, (ncols, n), NP[prec])
    y = crandn(rng, (ncols, m), NP[prec])
    ey = rel_err(to_host(op @ to_dev(x)), dense.apply(a, x))
    ez = rel_err(to_host(op.H @ to_dev(y)), dense.apply(a, y, True))
    assert ey <= tol and ez <= tol, (ey, ez)


def zoo(gpu, prec, rng):
    """(name, operator, dense matrix) for a few square structured operators."""
    dt = tdt(prec)
    c = (crandn(rng, 64, np.complex128) / 8).astype(NP[prec])
    c[0] += 4  # spectrum 4 + O(1): well conditioned, so the inverse checks stay tight
    d = ((1 + rng.random(64)) * np.exp(2j * np.pi * rng.random(64))).astype(NP[prec])
    g = crandn(rng, (8, 8), NP[prec])
    col, row = crandn(rng, 64, NP[prec]), crandn(rng, 64, NP[prec])
    perm = rng.permutation(64).astype(np.int32)
    C, D = gpu.Circulant(to_dev(c)), gpu.Diag(to_dev(d))
    F, H = gpu.Fourier(64, dt), gpu.Hadamard(64, dt)
    G, T = gpu.Dense(to_dev(g)), gpu.Toeplitz(to_dev(col), to_dev(row))
    S = gpu.SelectRows(64, to_dev(perm), dt)
    dC, dD, dF, dH = dense.circulant(c), dense.diag(d), dense.fourier(64), dense.hadamard(64)
    dG, dT, dS = g.astype(np.complex128), dense.toeplitz(col, row), dense.select_rows(64, perm)
    F8 = gpu.Fourier(8, dt)
    return [
        ("circulant", C, dC), ("diag", D, dD), ("fourier", F, dF), ("hadamard", H, dH), ("dense", G, dG),
        ("toeplitz", T, dT), ("permutation", S, dS),
        ("kron", gpu.Kron(F8, G), dense.kron(dense.fourier(8), dG)),
        ("kron_fc", gpu.Kron(F8, gpu.Circulant(to_dev(c[:8]))), dense.kron(dense.fourier(8), dense.circulant(c[:8]))),
        ("product", gpu.Product(C, D), dC @ dD),
        ("blkdiag", gpu.BlkDiag(C, D), dense.blkdiag(dC, dD)),
        ("adjoint", C.H, dC.conj().T),
        ("conj_of_circulant", C.conj, dC.conj()),
    ]


@pytest.mark.parametrize("prec", ["c64", "c128"])
def test_conj_and_transpose(gpu, prec):
    rng = np.random.default_rng(31)
    for name, op, a in zoo(gpu, prec, rng):
        check_both(op.conj, a.conj(), rng, prec)
        check_both(op.T, a.T, rng, prec)
    # accumulate path: a Sum of conj views
    name, op, a = zoo(gpu, prec, rng)[5]
    check_both(gpu.Sum(op.conj, op.conj), 2 * a.conj(), rng, prec)


@pytest.mark.parametrize("prec", ["c64", "c128"])
def test_gram(gpu, prec):
    rng = np.random.default_rng(37)
    for name, op, a in zoo(gpu, prec, rng):  # measured <= 4.7e-7 (c64), 1.1e-15 (c128)
        check_both(op.gram, a.conj().T @ a, rng, prec)
    n, rows = 32, np.array([1, 4, 9, 30], np.int32)
    S = gpu.SelectRows(n, to_dev(rows), tdt(prec))
    check_both(S.gram, dense.select_rows(n, rows).T @ dense.select_rows(n, rows), rng, prec)


@pytest.mark.parametrize("prec", ["c64", "c128"])
def test_structured_inverse(gpu, prec):
    import paper_1710_09578_amd as fm

    rng = np.random.default_rng(41)
    for name, op, a in zoo(gpu, prec, rng):  # condition numbers <= 5.2; measured <= 3.0e-7 (c64), 2.3e-15 (c128)
        if name == "toeplitz":
            continue  # Levinson: test_toeplitz_inverse_levinson
        if name in ("dense", "kron"):
            with pytest.raises(fm.FmError) as e:
                op.inverse
            assert e.value.code == "FM_E_UNSUPPORTED"
            continue
        check_both(op.inverse, np.linalg.inv(a), rng, prec)
    with pytest.raises(fm.FmError) as e:  # singular circulant: c = ones has c_hat = (n, 0, ..., 0)
        gpu.Circulant(to_dev(np.ones(16, NP[prec]))).inverse
    assert e.value.code == "FM_E_INVALID"
    with pytest.raises(fm.FmError) as e:
        gpu.Dense(to_dev(crandn(rng, (4, 6), NP[prec]))).inverse
    assert e.value.code == "FM_E_SHAPE"


@pytest.mark.parametrize("prec", ["c64", "c128"])
@pytest.mark.parametrize("n", [3, 5, 12, 100, 1000, 3001])
def test_fourier_any_size(gpu, prec, n):
    rng = np.random.default_rng(n)
    F = gpu.Fourier(n, tdt(prec))
    check_both(F, dense.fourier(n), rng, prec)
    if n <= 100:
        check_both(gpu.Kron(F, gpu.Fourier(8, tdt(prec))), dense.kron(dense.fourier(n), dense.fourier(8)), rng, prec)
        check_both(F.inverse, np.linalg.inv(dense.fourier(n)), rng, prec)


@pytest.mark.parametrize("prec", ["c64", "c128"])
@pytest.mark.parametrize("n", [3, 100, 1000, 5000])
def test_circulant_any_size(gpu, prec, n):
    rng = np.random.default_rng(n + 1)
    c = crandn(rng, n, NP[prec])
    check_both(gpu.Circulant(to_dev(c)), dense.circulant(c), rng, prec)


@pytest.mark.parametrize("prec", ["c64", "c128"])
@pytest.mark.parametrize("order,taps", [(4, 0b0011), (10, 0b1001), (12, 0b1010011)])
def test_lfsr_circulant(gpu, prec, order, taps):
    rng = np.random.default_rng(order)
    op = gpu.LFSRCirculant(order, taps, 1, tdt(prec))
    check_both(op, dense.circulant(dense.lfsr_sequence(order, taps, 1)), rng, prec)


@pytest.mark.parametrize("prec", ["c64", "c128"])
@pytest.mark.parametrize("n", [1, 7, 100, 1500])
def test_toeplitz_inverse_levinson(gpu, prec, n):
    """Square Toeplitz inverse applied by Levinson recursion (forward and
    adjoint), with a well-conditioned generator; the accumulate path through a
    Sum; a zero diagonal (singular first leading minor) gives NaN."""
    rng = np.random.default_rng(n + 7)
    col = (crandn(rng, n, np.complex128) / np.sqrt(n)).astype(NP[prec])
    row = (crandn(rng, n, np.complex128) / np.sqrt(n)).astype(NP[prec])
    col[0] += 3
    T = gpu.Toeplitz(to_dev(col), to_dev(row))
    inv = np.linalg.inv(dense.toeplitz(col, row))
    # the recursion runs n dependent steps in the working precision, so its
    # rounding grows with n: measured 1.7e-5 at n = 1500 in complex64
    # (condition number 9) and 4.3e-15 in complex128
    tol = {"c64": 1e-4, "c128": 1e-12}[prec]
    check_both(T.inverse, inv, rng, prec, tol=tol)
    check_both(gpu.Sum(T.inverse, T.inverse), 2 * inv, rng, prec, tol=tol)
    if n > 1:
        col0 = col.copy()
        col0[0] = 0
        y = to_host(gpu.Toeplitz(to_dev(col0), to_dev(row)).inverse @ to_dev(crandn(rng, (1, n), NP[prec])))
        assert np.all(np.isnan(y))


@pytest.mark.parametrize("prec", ["c64", "c128"])
def test_calibrated_path(gpu, prec):
    """Run-time calibration between the structured transforms and the dense
    product: whichever path it keeps, and each path when forced, matches the
    oracle; operators above 64 x 64 are refused."""
    import paper_1710_09578_amd as fm

    rng = np.random.default_rng(43)
    dt = tdt(prec)
    c = crandn(rng, 16, NP[prec])
    col, row = crandn(rng, 24, NP[prec]), crandn(rng, 20, NP[prec])
    rows = np.array([0, 3, 5, 9, 12, 15], np.int32)
    cases = [
        (gpu.Circulant(to_dev(c)), dense.circulant(c)),
        (gpu.Toeplitz(to_dev(col), to_dev(row)), dense.toeplitz(col, row)),
        (gpu.Fourier(32, dt), dense.fourier(32)),
        (gpu.Kron(gpu.Fourier(4, dt), gpu.Hadamard(8, dt)), dense.kron(dense.fourier(4), dense.hadamard(8))),
        (gpu.Product(gpu.SelectRows(16, to_dev(rows), dt), gpu.Circulant(to_dev(c))),
         dense.select_rows(16, rows) @ dense.circulant(c)),
    ]
    for op, a in cases:
        info = op.calibrate(4096)
        assert info["path"] in ("dense", "structured") and info["ms_dense"] > 0 and info["ms_structured"] > 0
        check_both(op, a, rng, prec, ncols=300)
        for path in ("dense", "structured"):
            op.set_path(path)
            check_both(op, a, rng, prec, ncols=300)
            check_both(gpu.Sum(op, op), 2 * a, rng, prec)
    with pytest.raises(fm.FmError) as e:
        gpu.Fourier(128, dt).calibrate(16)
    assert e.value.code == "FM_E_UNSUPPORTED"


def test_dense_matrix_cores_every_shape(gpu):
    """The complex64 dense product on the matrix cores (64 vectors or more)
    for every padded shape 16/32/64 in and out, forward and adjoint, with
    strided columns, a ragged last work-group, and accumulation; against the
    FP64 product."""
    rng = np.random.default_rng(77)
    for m, n in ((5, 7), (16, 16), (20, 33), (33, 20), (64, 64), (48, 12), (1, 64), (64, 1)):
        a = crandn(rng, (n, m)).T.copy()  # m x n
        A = gpu.Dense(to_dev(a))
        for adj in (False, True):
            rin, rout = (m, n) if adj else (n, m)
            x = crandn(rng, (200, rin))
            y = to_host(A.apply(to_dev(x), adjoint=adj))
            assert rel_err(y, dense.apply(a, x, adj)) <= TOL["c64"], (m, n, adj)
        # accumulation through a Sum of the same operator
        x = crandn(rng, (130, n))
        y = to_host(gpu.Sum(A, A).apply(to_dev(x)))
        assert rel_err(y, 2 * dense.apply(a, x)) <= TOL["c64"], (m, n)


def test_calibration_model(gpu):
    """The device's calibration model: measured once over its grid (three
    classes, two dtypes, 5 sizes, 5 column counts), exported and loaded back,
    consulted by handles without timing them; a synthetic model checks the
    interpolation between grid points and the clamping outside the grid."""
    import paper_1710_09578_amd as fm

    table = fm.calibration_build()
    assert len(table) == 150 and all(e["ms_fast"] > 0 and e["ms_dense"] > 0 for e in table)
    fm.calibration_load(table)
    assert fm.calibration_table() == table
    rng = np.random.default_rng(5)
    # at a grid point the decision is the measured one
    for e in table[:10]:
        if e["dt"] != 1 or e["cls"] != 0:
            continue
        c = crandn(rng, e["n"])
        C = gpu.Circulant(to_dev(c))
        want = "dense" if e["ms_dense"] < e["ms_fast"] else "structured"
        assert C.choose_path(e["ncols"]) == want
        check_both(C, dense.circulant(c), rng, "c64", ncols=70)
    # synthetic model: dense faster by 2x at n <= 16 and ncols <= 16, slower elsewhere
    syn = []
    for cls in (0, 1, 2):
        for dt in (1, 2):
            for n in (8, 16, 32, 48, 64):
                for nc in (1, 16, 256, 4096, 65536):
                    fast = 1.0
                    dense_t = 0.5 if (n <= 16 and nc <= 16) else 2.0
                    syn.append({"cls": cls, "dt": dt, "n": n, "ncols": nc, "ms_fast": fast, "ms_dense": dense_t})
    fm.calibration_load(syn)
    col, row = crandn(rng, 12), crandn(rng, 12)
    T = gpu.Toeplitz(to_dev(col), to_dev(row))
    assert T.choose_path(4) == "dense"            # inside the dense corner
    check_both(T, dense.toeplitz(col, row), rng, "c64", ncols=80)
    assert T.choose_path(100000) == "structured"  # clamped to 65536
    assert T.choose_path(64) == "structured"      # log2 64 halfway between 16 and 256: ratio 0, ties keep structured
    assert T.choose_path(31) == "dense"           # log2 31 nearer 16: negative ratio
    F = gpu.Fourier(64)
    assert F.choose_path(1) == "structured"
    with pytest.raises(fm.FmError):
        gpu.Product(gpu.Circulant(to_dev(crandn(rng, 8))), gpu.Circulant(to_dev(crandn(rng, 8)))).choose_path(16)
    fm.calibration_load(table)
