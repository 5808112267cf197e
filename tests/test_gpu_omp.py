"""GPU parity of orthogonal matching pursuit (fm_omp) against the FP64 oracle.

The greedy choice is an argmax taken in the kernel's precision, so the
selections are compared exactly over the steps where the oracle's two largest
correlations are separated by more than that precision's error (every step of
the true support here; see separated_steps), and x is compared with the
oracle's least-squares solution on the support the GPU chose (unique for a
full-rank A_S), column by column (relative L2 <= 2e-5 complex64, <= 1e-12
complex128).
"""

import numpy as np
import pytest

from oracle import dense, omp
from tests.gpu_util import TOL, crandn, rel_err, to_dev, to_host

pytestmark = pytest.mark.gpu

NP = {"c64": np.complex64, "c128": np.complex128}


def tdt(prec):
    import torch

    return {"c64": torch.complex64, "c128": torch.complex128}[prec]


def cs_problem(gpu, prec, n=1024, m=256, k=12, ncols=3, seed=0, sigma=1e-3):
    rng = np.random.default_rng(seed)
    c = crandn(rng, n, NP[prec])
    rows = np.sort(rng.choice(n, m, replace=False)).astype(np.int32)
    a = dense.product(dense.select_rows(n, rows), dense.circulant(c))
    xt = np.zeros((ncols, n), np.complex128)
    for j in range(ncols):
        xt[j, rng.choice(n, k, replace=False)] = np.sign(rng.standard_normal(k)) * (1 + rng.random(k))
    b = (dense.apply(a, xt) + sigma * crandn(rng, (ncols, m), np.complex128)).astype(NP[prec])
    A = gpu.Product(gpu.SelectRows(n, to_dev(rows), tdt(prec)), gpu.Circulant(to_dev(c)))
    return A, a, b, xt


# Unit roundoff of the working precision. A residual r = b - A x computed in
# it carries an error of about u ||b||, i.e. u ||b|| / ||r|| relative to r:
# small while the true support is being found, ~1e-4 in complex64 once r is
# at noise level 1e-3. Where the oracle's two largest unchosen |A^H r| lie
# closer than 64 times that (relative to the largest), either choice is a
# correct OMP step in the working precision.
UNIT = {"c64": 2.0 ** -24, "c128": 2.0 ** -53}


def separated_steps(a, b, sup_ref, atoms, u):
    """Leading steps of the oracle's run on one column whose choice is
    separated by more than 64 u ||b|| / ||r|| (compared exactly); the rest
    are checked for validity only."""
    r = b.astype(np.complex128)
    bn = np.linalg.norm(r)
    chosen = []
    for step in range(atoms):
        c = np.abs(a.conj().T @ r)
        c[chosen] = -1.0
        top = np.sort(c)[::-1]
        if top[0] - top[1] <= 64 * u * bn / np.linalg.norm(r) * top[0]:
            return step
        chosen.append(int(sup_ref[step]))
        xs = np.linalg.lstsq(a[:, chosen], b, rcond=None)[0]
        r = b - a[:, chosen] @ xs
    return atoms


def check_selections(a, b, sup, sup_ref, atoms_ref, xh, x_ref, prec, min_steps):
    """Selections equal to the oracle's over its separated steps (at least
    min_steps of them); x equal to the oracle's where the whole run is
    separated; everywhere x is the least-squares solution on the GPU's own
    support."""
    for j in range(b.shape[0]):
        t = separated_steps(a, b[j], sup_ref[j], int(atoms_ref[j]), UNIT[prec])
        assert t >= min(min_steps, int(atoms_ref[j])), f"column {j}: the oracle's run is not separated at step {t}"
        assert np.array_equal(sup[j][:t], sup_ref[j][:t]), (j, t, sup[j], sup_ref[j])
        if t == atoms_ref[j]:
            assert rel_err(xh[j:j + 1], x_ref[j:j + 1]) <= TOL[prec]
        assert rel_err(xh[j], omp.least_squares_on(a, b[j], sup[j])) <= TOL[prec]


@pytest.mark.parametrize("prec", ["c64", "c128"])
@pytest.mark.parametrize("k", [1, 5, 12, 20])
@pytest.mark.parametrize("m", [256, 768])
def test_omp_matches_oracle(gpu, prec, k, m):
    """m = 256: one work-group per column for the Gram-Schmidt step; m = 768:
    the step split over three work-groups per column. The selections are
    compared with the oracle's over its separated steps (every step of the
    true support, and those after it whose two largest correlations differ
    by more than the working precision's error); a column whose run is
    separated throughout gives the oracle's x."""
    A, a, b, _ = cs_problem(gpu, prec, m=m)
    x_ref, sup_ref, atoms_ref = omp.omp(a, b, k)
    x, sup, st = gpu.omp(A, to_dev(b), k)
    sup = to_host(sup)
    assert [s["atoms"] for s in st] == list(atoms_ref) and all(s["status"] == 0 for s in st)
    xh = to_host(x)
    check_selections(a, b, sup, sup_ref, atoms_ref, xh, x_ref, prec, 12)  # 12: the true support
    for j in range(b.shape[0]):
        assert rel_err(xh[j], omp.least_squares_on(a, b[j], sup[j])) <= TOL[prec]
        res = np.linalg.norm(dense.apply(a, xh[j:j + 1])[0] - b[j])
        assert abs(st[j]["res_norm"] - res) <= 1e-3 * max(res, 1e-3 * np.linalg.norm(b[j]))


@pytest.mark.parametrize("prec", ["c64", "c128"])
@pytest.mark.parametrize("m", [192, 640])
def test_omp_recovers_support_and_stops_on_tolerance(gpu, prec, m):
    """Noiseless sparse vectors: the tolerance ends each column after exactly
    its own sparsity (uneven across columns); m = 640 takes the split
    Gram-Schmidt step."""
    rng = np.random.default_rng(3)
    n = 1024 if m > 512 else 512
    c = crandn(rng, n, NP[prec])
    rows = np.sort(rng.choice(n, m, replace=False)).astype(np.int32)
    a = dense.product(dense.select_rows(n, rows), dense.circulant(c))
    ks = [2, 7, 4]
    xt = np.zeros((3, n), np.complex128)
    for j, kk in enumerate(ks):
        xt[j, rng.choice(n, kk, replace=False)] = 1 + rng.random(kk)
    b = dense.apply(a, xt).astype(NP[prec])
    A = gpu.Product(gpu.SelectRows(n, to_dev(rows), tdt(prec)), gpu.Circulant(to_dev(c)))
    tol = 1e-4 if prec == "c64" else 1e-10
    x, sup, st = gpu.omp(A, to_dev(b), 16, tol=tol)
    x_ref, sup_ref, atoms_ref = omp.omp(a, b, 16, tol=tol)
    assert [s["atoms"] for s in st] == ks == list(atoms_ref)
    assert np.array_equal(to_host(sup), sup_ref)
    assert rel_err(to_host(x), xt) <= (1e-5 if prec == "c64" else 1e-11)


@pytest.mark.parametrize("prec", ["c64", "c128"])
@pytest.mark.parametrize("rows", [8, 600])
def test_omp_dependent_atom_stops(gpu, prec, rows):
    """Columns 0 and 1 of A are equal: once the other columns are used up the
    only candidate left depends on the chosen ones; the column stops with
    status 2 and keeps its independent atoms (600 rows: the Gram-Schmidt step
    split over work-groups)."""
    rng = np.random.default_rng(5)
    d = crandn(rng, (rows, 4), NP[prec])
    d[:, 1] = d[:, 0]
    b = crandn(rng, (1, rows), NP[prec])
    x, sup, st = gpu.omp(gpu.Dense(to_dev(d)), to_dev(b), 4)
    assert st[0]["status"] == 2 and st[0]["atoms"] == 3
    s = to_host(sup)[0]
    assert s[3] == -1 and len(set(s[:3].tolist()) & {0, 1}) == 1
    assert rel_err(to_host(x), omp.least_squares_on(d, b[0], s)[None, :]) <= TOL[prec]


@pytest.mark.parametrize("prec", ["c64", "c128"])
@pytest.mark.parametrize("ncols", [5, 130])
def test_omp_column_counts(gpu, prec, ncols):
    """Few columns take the Gram-Schmidt step split over several work-groups
    per column, many columns one work-group each: both against the oracle."""
    A, a, b, _ = cs_problem(gpu, prec, n=1024, m=600, k=6, ncols=ncols, seed=9)
    x_ref, sup_ref, atoms_ref = omp.omp(a, b, 8)
    x, sup, st = gpu.omp(A, to_dev(b), 8)
    assert [s["atoms"] for s in st] == list(atoms_ref)
    check_selections(a, b, to_host(sup), sup_ref, atoms_ref, to_host(x), x_ref, prec, 6)  # 6: the true support


@pytest.mark.parametrize("prec", ["c64", "c128"])
@pytest.mark.parametrize("shape,select", [((600, 400), True), ((300, 500), False), ((5000, 5000), True)])
def test_omp_toeplitz_columns_from_the_generator(gpu, prec, shape, select):
    """OMP on T and S T with T a Toeplitz (power-of-two and 4096 * 3
    embeddings): the chosen columns come from the stored embedded generator,
    T[i, j] = g[(i - j) mod L]; selections and x against the oracle."""
    rng = np.random.default_rng(sum(shape) + select)
    mt, n = shape
    col, row = crandn(rng, mt, NP[prec]), crandn(rng, n, NP[prec])
    T = gpu.Toeplitz(to_dev(col), to_dev(row))
    a = dense.toeplitz(col, row)
    A = T
    if select:
        rows = np.sort(rng.choice(mt, mt // 3, replace=False)).astype(np.int32)
        A = gpu.Product(gpu.SelectRows(mt, to_dev(rows), tdt(prec)), T)
        a = dense.select_rows(mt, rows) @ a
    k_true, k = 5, 7
    xt = np.zeros((2, n), np.complex128)
    for j in range(2):
        xt[j, rng.choice(n, k_true, replace=False)] = np.sign(rng.standard_normal(k_true)) * (1 + rng.random(k_true))
    b = (dense.apply(a, xt) + 1e-3 * crandn(rng, (2, a.shape[0]), np.complex128)).astype(NP[prec])
    x_ref, sup_ref, atoms_ref = omp.omp(a, b, k)
    x, sup, st = gpu.omp(A, to_dev(b), k)
    assert [s["atoms"] for s in st] == list(atoms_ref)
    check_selections(a, b, to_host(sup), sup_ref, atoms_ref, to_host(x), x_ref, prec, k_true)


@pytest.mark.parametrize("prec", ["c64", "c128"])
@pytest.mark.parametrize("ncols", [1, 2])
def test_omp_select_toeplitz_long_embedding(gpu, prec, ncols):
    """S T with T a 60000 x 2000 Toeplitz (embedding L = 65536) and S 1500
    of its rows: with one or two columns the correlations A^H r run with
    1024-point rows. Selections and x against the oracle on the dense
    selected rows, T[i, j] = col[i - j] (i >= j) or row[j - i]."""
    rng = np.random.default_rng(41 + ncols)
    mt, n = 60000, 2000
    col, row = crandn(rng, mt, NP[prec]), crandn(rng, n, NP[prec])
    row[0] = col[0]
    T = gpu.Toeplitz(to_dev(col), to_dev(row))
    assert T.transform_length == 65536
    rows = np.sort(rng.choice(mt, 1500, replace=False)).astype(np.int32)
    A = gpu.Product(gpu.SelectRows(mt, to_dev(rows), tdt(prec)), T)
    d = rows.astype(np.int64)[:, None] - np.arange(n)[None, :]
    a = np.where(d >= 0, col.astype(np.complex128)[np.clip(d, 0, None)],
                 row.astype(np.complex128)[np.clip(-d, 0, None)])
    k_true, k = 5, 7
    xt = np.zeros((ncols, n), np.complex128)
    for j in range(ncols):
        xt[j, rng.choice(n, k_true, replace=False)] = np.sign(rng.standard_normal(k_true)) * (1 + rng.random(k_true))
    b = (dense.apply(a, xt) + 1e-3 * crandn(rng, (ncols, a.shape[0]), np.complex128)).astype(NP[prec])
    x_ref, sup_ref, atoms_ref = omp.omp(a, b, k)
    x, sup, st = gpu.omp(A, to_dev(b), k)
    assert [s["atoms"] for s in st] == list(atoms_ref)
    check_selections(a, b, to_host(sup), sup_ref, atoms_ref, to_host(x), x_ref, prec, k_true)


@pytest.mark.parametrize("prec", ["c64", "c128"])
def test_omp_split_argmax(gpu, prec):
    """n = 16384 with two columns: the argmax runs over four work-groups per
    column and a combining launch (first index on ties across the ranges);
    a duplicated column must pick the same atoms as its twin."""
    A, a, b, _ = cs_problem(gpu, prec, n=16384, m=1024, k=8, ncols=2, seed=13)
    b = np.concatenate([b, b[:1]])
    x_ref, sup_ref, atoms_ref = omp.omp(a, b, 10)
    x, sup, st = gpu.omp(A, to_dev(b), 10)
    sup, xh = to_host(sup), to_host(x)
    assert [s["atoms"] for s in st] == list(atoms_ref)
    check_selections(a, b, sup, sup_ref, atoms_ref, xh, x_ref, prec, 8)
    assert np.array_equal(sup[0], sup[2]) and np.array_equal(xh[0], xh[2])


@pytest.mark.parametrize("prec", ["c64", "c128"])
@pytest.mark.parametrize("m", [256, 768])
def test_omp_zero_and_trivial_inputs(gpu, prec, m):
    A, a, b, _ = cs_problem(gpu, prec, m=m, ncols=2)
    b = b.copy()
    b[1] = 0
    x, sup, st = gpu.omp(A, to_dev(b), 6)
    assert st[1]["atoms"] == 0 and np.all(to_host(x)[1] == 0) and np.all(to_host(sup)[1] == -1)
    x, sup, st = gpu.omp(A, to_dev(b), 6, tol=1.0)  # tol >= 1: nothing to do
    assert all(s["atoms"] == 0 for s in st) and np.all(to_host(x) == 0)


def test_omp_compressed_sensing_full_size(gpu):
    """N = 65536, M = 4096 rows of a Rademacher circulant, 64-sparse truth,
    noise 1e-3, 64 atoms (complex64). The support is recovered exactly; x is
    compared with the least-squares solution on it, whose 4096 x 64 columns
    are built from the circulant's definition."""
    from workloads import compressed_sensing_65536

    w = compressed_sensing_65536()
    c, rows, xt = w["c"], w["rows"], w["x_true"]
    n = c.size
    A = gpu.Product(gpu.SelectRows(n, to_dev(rows)), gpu.Circulant(to_dev(c)))

    def columns(js):  # (S C(c))[:, j] = c[(rows - j) mod n], from the definition
        return np.stack([c.astype(np.complex128)[(rows - j) % n] for j in js], axis=1)

    truth = np.nonzero(xt[0])[0]
    bh = (columns(truth) @ xt[0, truth] + w["noise"][0]).astype(np.complex64)
    x, sup, st = gpu.omp(A, to_dev(bh[None, :]), 64)
    s = to_host(sup)[0]
    assert sorted(s.tolist()) == sorted(truth.tolist())
    xs = np.linalg.lstsq(columns(s), bh.astype(np.complex128), rcond=None)[0]
    ref = np.zeros(n, np.complex128)
    ref[s] = xs
    err = rel_err(to_host(x), ref[None, :])
    print(f"omp N=65536 M=4096 K=64: support recovered, x rel err {err:.2e}, status {st[0]}")
    assert err <= TOL["c64"]
