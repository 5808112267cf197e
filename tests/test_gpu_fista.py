"""GPU parity of the solver (fm_fista) and the FP64 power iteration
(fm_power_iteration) against the oracle.

The same step constant L and regularisation weights are given to both sides
(the oracle computes them in FP64); the iterates after K steps are compared
column by column (relative L2 <= 2e-5 for complex64, <= 1e-12 for
complex128). The power iteration runs in FP64 on the GPU whatever the
operator's dtype and must match the oracle's run from the same start vector
to 1e-12 relative.
"""

import numpy as np
import pytest

from oracle import dense, fista, structured
from tests.gpu_util import TOL, crandn, rel_err, to_dev, to_host

pytestmark = pytest.mark.gpu

NP = {"c64": np.complex64, "c128": np.complex128}


def tdt(prec):
    import torch

    return {"c64": torch.complex64, "c128": torch.complex128}[prec]


def cs_problem(gpu, prec, n=1024, m=256, k=16, ncols=3, seed=0):
    """Row-selected circulant with sparse truths and noisy measurements."""
    rng = np.random.default_rng(seed)
    c = crandn(rng, n, NP[prec])
    rows = np.sort(rng.choice(n, m, replace=False)).astype(np.int32)
    a = dense.product(dense.select_rows(n, rows), dense.circulant(c))
    xt = np.zeros((ncols, n), np.complex128)
    for j in range(ncols):
        xt[j, rng.choice(n, k, replace=False)] = rng.standard_normal(k)
    b = (dense.apply(a, xt) + 1e-3 * crandn(rng, (ncols, m), np.complex128)).astype(NP[prec])
    A = gpu.Product(gpu.SelectRows(n, to_dev(rows), tdt(prec)), gpu.Circulant(to_dev(c)))
    return A, a, b


# ---------------------------------------------------------------- power iteration
@pytest.mark.parametrize("kind", ["circulant", "toeplitz", "select_circulant", "kron_c128"])
def test_power_iteration_matches_oracle(gpu, kind):
    import torch

    rng = np.random.default_rng(7)
    if kind == "circulant":
        c = crandn(rng, 256)
        A, a = gpu.Circulant(to_dev(c)), dense.circulant(c)
    elif kind == "toeplitz":
        col, row = crandn(rng, 300), crandn(rng, 200)
        A, a = gpu.Toeplitz(to_dev(col), to_dev(row)), dense.toeplitz(col, row)
    elif kind == "select_circulant":
        A, a, _ = cs_problem(gpu, "c64")
    else:
        g = crandn(rng, (5, 3), np.complex128)
        A = gpu.Kron(gpu.Fourier(8, torch.complex128), gpu.Dense(to_dev(g)))
        a = dense.kron(dense.fourier(8), g)
    v0 = crandn(rng, a.shape[1], np.complex128)
    L_ref, it_ref = fista.power_iteration(a, v0, max_iters=300, tol=1e-13)
    L, it = gpu.power_iteration(A, to_dev(v0), max_iters=300, tol=1e-13)
    assert abs(L - L_ref) <= 1e-12 * L_ref
    assert abs(it - it_ref) <= 1
    # the default SplitMix64 start vector, drawn independently on each side
    L2_ref, _ = fista.power_iteration(a, fista.splitmix64_start(a.shape[1], 11), max_iters=300, tol=1e-13)
    L2, _ = gpu.power_iteration(A, None, seed=11, max_iters=300, tol=1e-13)
    assert abs(L2 - L2_ref) <= 1e-12 * L2_ref


@pytest.mark.parametrize("kind", ["toeplitz", "select_circulant"])
def test_power_iteration_chunk_boundaries(gpu, kind):
    """The estimate after exactly k iterations (tol 0) around the chunk
    boundaries of 16: the first chunk launched directly, later full chunks
    replayed from one captured graph, the remainder launched directly."""
    rng = np.random.default_rng(19)
    if kind == "toeplitz":
        col, row = crandn(rng, 300), crandn(rng, 200)
        A, a = gpu.Toeplitz(to_dev(col), to_dev(row)), dense.toeplitz(col, row)
    else:
        A, a, _ = cs_problem(gpu, "c64", seed=3)
    v0 = crandn(rng, a.shape[1], np.complex128)
    for k in (1, 15, 16, 17, 32, 33, 48, 63):
        L_ref, it_ref = fista.power_iteration(a, v0, max_iters=k, tol=0.0)
        L, it = gpu.power_iteration(A, to_dev(v0), max_iters=k, tol=0.0)
        if it_ref == k:  # (the oracle stops early only where two estimates are equal)
            assert it == k, (k, it)
        assert abs(L - L_ref) <= 1e-12 * L_ref, (k, L, L_ref)
        L2, _ = gpu.power_iteration(A, to_dev(v0), max_iters=k, tol=0.0)
        assert L2 == L, k  # a second call, with its own graph, gives the same bits


@pytest.mark.parametrize("kind", ["circulant_65536", "toeplitz_30000", "circulant_1048576"])
def test_power_iteration_select_long(gpu, kind):
    """Row-selected convolutions of power-of-two length L >= 65536, whose
    products run through the solver's passes with 1024-point rows: the
    estimate after exactly k iterations (tol 0) against the oracle's run
    with FFT64 products from the same start vector."""
    rng = np.random.default_rng(23)
    if kind.startswith("circulant"):
        n = int(kind.split("_")[1])
        c = crandn(rng, n)
        rows = np.sort(rng.choice(n, n // 16, replace=False)).astype(np.int32)
        ap, ad = structured.select_circulant_fft64(c.astype(np.complex128), rows)
        C = gpu.Circulant(to_dev(c))
    else:
        n = 30000
        col, row = crandn(rng, n), crandn(rng, n)
        rows = np.sort(rng.choice(n, n // 4, replace=False)).astype(np.int32)
        t_ap = lambda v: structured.toeplitz_apply_fft64(col, row, v, L=65536)
        t_ad = lambda v: structured.toeplitz_apply_fft64(col, row, v, True, L=65536)
        ap = lambda v: t_ap(v)[:, rows]

        def ad(u):
            z = np.zeros((u.shape[0], n), np.complex128)
            z[:, rows] = u
            return t_ad(z)
        C = gpu.Toeplitz(to_dev(col), to_dev(row))
        assert C.transform_length == 65536
    A = gpu.Product(gpu.SelectRows(n, to_dev(rows)), C)
    v0 = crandn(rng, n, np.complex128)
    for k in ((1, 17, 40) if n <= 65536 else (1, 5)):
        L_ref, _ = fista.power_iteration_op(lambda v: ap(v[None])[0], lambda u: ad(u[None])[0], v0, k, 0.0)
        L, it = gpu.power_iteration(A, to_dev(v0), max_iters=k, tol=0.0)
        assert it == k
        assert abs(L - L_ref) <= 1e-12 * L_ref, (kind, k, L, L_ref)


# ---------------------------------------------------------------- FISTA / ISTA
@pytest.mark.parametrize("prec", ["c64", "c128"])
@pytest.mark.parametrize("momentum", [True, False])
@pytest.mark.parametrize("iters", [1, 7, 60])
def test_fista_matches_oracle(gpu, prec, momentum, iters):
    A, a, b = cs_problem(gpu, prec)
    L = fista.spectral_norm_sq(a)
    lam = fista.lambda_rule(a, b, 0.05)
    x_ref, _ = fista.fista(a, b, lam, L, iters, momentum=momentum)
    xs = []
    for j in range(b.shape[0]):  # lam_abs is per call: one column at a time
        x, st = gpu.fista(A, to_dev(b[j:j + 1]), iters=iters, momentum=momentum, lam=lam[j], L=L)
        assert st[0]["iters"] == iters and st[0]["status"] == 0
        xs.append(to_host(x)[0])
    assert rel_err(np.stack(xs), x_ref) <= TOL[prec]


@pytest.mark.parametrize("prec", ["c64", "c128"])
def test_lambda_rule_and_block_solve(gpu, prec):
    """lam_j = 0.05 ||A^H b_j||_inf computed on the GPU per column; a block of
    columns solved in one call."""
    A, a, b = cs_problem(gpu, prec, ncols=5, seed=3)
    L = fista.spectral_norm_sq(a)
    lam = fista.lambda_rule(a, b, 0.05)
    x, st = gpu.fista(A, to_dev(b), iters=40, lam_rel=0.05, L=L)
    got = np.array([s["lam"] for s in st])
    assert np.all(np.abs(got - lam) <= (1e-5 if prec == "c64" else 1e-13) * lam)
    x_ref, _ = fista.fista(a, b, got, L, 40)  # same weights on both sides
    assert rel_err(to_host(x), x_ref) <= TOL[prec]


def test_zero_iterations_and_large_lambda(gpu):
    A, a, b = cs_problem(gpu, "c64")
    L = fista.spectral_norm_sq(a)
    x0 = crandn(np.random.default_rng(1), (3, a.shape[1]))
    x, st = gpu.fista(A, to_dev(b), iters=0, lam=1.0, L=L, x0=to_dev(x0))
    assert np.array_equal(to_host(x), x0) and all(s["iters"] == 0 for s in st)
    lam_max = float(np.max(fista.lambda_rule(a, b, 1.0)))
    x, _ = gpu.fista(A, to_dev(b), iters=25, lam=lam_max * 1.0001, L=L)
    assert np.count_nonzero(to_host(x)) == 0


def test_warm_start(gpu):
    A, a, b = cs_problem(gpu, "c128", seed=5)
    L = fista.spectral_norm_sq(a)
    lam = float(fista.lambda_rule(a, b[:1], 0.05)[0])
    x0 = crandn(np.random.default_rng(2), (1, a.shape[1]), np.complex128)
    x, _ = gpu.fista(A, to_dev(b[:1]), iters=10, lam=lam, L=L, x0=to_dev(x0))
    x_ref, _ = fista.fista(a, b[:1], lam, L, 10, x0=x0)
    assert rel_err(to_host(x), x_ref) <= TOL["c128"]


def test_stop_rule_iteration_counts(gpu):
    A, a, b = cs_problem(gpu, "c128", ncols=4, seed=9)
    L = fista.spectral_norm_sq(a)
    lam = 0.05 * float(np.max(fista.lambda_rule(a, b, 1.0)))
    x, st = gpu.fista(A, to_dev(b), iters=400, lam=lam, L=L, stop_tol=1e-5)
    x_ref, done = fista.fista(a, b, lam, L, 400, stop_tol=1e-5)
    counts = np.array([s["iters"] for s in st])
    assert np.all(np.abs(counts - done) <= 1) and np.all(done < 400)
    for j in range(4):  # each frozen column equals the plain run to its own count
        xj, _ = fista.fista(a, b[j:j + 1], lam, L, int(counts[j]))
        assert rel_err(to_host(x)[j:j + 1], xj) <= 1e-12


def test_non_finite_column_is_frozen(gpu):
    A, a, b = cs_problem(gpu, "c64", ncols=3, seed=4)
    L = fista.spectral_norm_sq(a)
    bad = b.copy()
    bad[1, 5] = np.nan
    x, st = gpu.fista(A, to_dev(bad), iters=20, lam=0.1, L=L)
    assert st[1]["status"] == 1 and st[0]["status"] == 0 and st[2]["status"] == 0
    x_ref, _ = fista.fista(a, b[[0, 2]], 0.1, L, 20)
    assert rel_err(to_host(x)[[0, 2]], x_ref) <= TOL["c64"]


# ---------------------------------------------------------------- compressed-sensing configuration
@pytest.mark.parametrize("prec", ["c64", "c128"])
def test_compressed_sensing_65536(gpu, prec):
    """Row-selected Rademacher circulant, N = 65536, M = 4096, 64-sparse truth,
    sigma = 1e-3, 200 FISTA iterations, lam = 0.05 ||A^H b||_inf. Oracle:
    the same iteration with FFT64 products (pinned to the dense form)."""
    import torch

    from workloads import compressed_sensing_65536

    d = compressed_sensing_65536()
    c, rows, xt, noise = d["c"], d["rows"], d["x_true"], d["noise"]
    ap, ad = structured.select_circulant_fft64(c, rows)
    b = (ap(xt.astype(np.complex128)) + noise).astype(NP[prec])
    L_ref, _ = fista.power_iteration_op(lambda v: ap(v[None])[0], lambda u: ad(u[None])[0],
                                        fista.splitmix64_start(65536, 0), 500, 1e-13)
    lam = fista.lambda_rule_op(ad, b, 0.05)
    A = gpu.Product(gpu.SelectRows(65536, to_dev(rows), tdt(prec)),
                    gpu.Circulant(to_dev(c.astype(NP[prec]))))
    L_gpu, _ = gpu.power_iteration(A, None, seed=0, max_iters=500, tol=1e-13)
    assert abs(L_gpu - L_ref) <= 1e-12 * L_ref
    x, st = gpu.fista(A, to_dev(b), iters=200, lam=float(lam[0]), L=L_ref)
    x_ref, _ = fista.fista_op(ap, ad, 65536, b, lam, L_ref, 200)
    err = rel_err(to_host(x), x_ref)
    print(f"compressed sensing {prec}: rel err after 200 iterations {err:.3e}")
    assert err <= TOL[prec]
