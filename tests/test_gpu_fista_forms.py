"""The per-operator solver (fm_fista) on every form of its fused iteration:
A = C and A = S C with C a circulant or Toeplitz operator whose embedding is
a single pass (L <= 4096), a four-step length with the strided factor folded
into the row pass (n2 <= 8), or a separate strided pass (n2 > 8), for
power-of-two and mixed lengths (one- and two-thread strided columns), in
complex64 and complex128, FISTA and ISTA, several columns. The oracle runs
the same iteration in FP64 with FFT64 products of any cyclic length >=
M + N - 1 (pinned to the dense form), from the same L and lambda (computed by
the oracle), and the iterates after K steps must match per column (2e-5 /
1e-12). An operator of another form (a Diag in the product) goes through the
general loop and must match as well."""

import numpy as np
import pytest

from oracle import fista, structured
from tests.gpu_util import TOL, crandn, rel_err, to_dev, to_host

pytestmark = pytest.mark.gpu

NP = {"c64": np.complex64, "c128": np.complex128}


def tdt(prec):
    import torch

    return {"c64": torch.complex64, "c128": torch.complex128}[prec]


def p2(v):
    return 1 << int(np.ceil(np.log2(v)))


# (N, expected embedding length L, strided factor) -- square Toeplitz N x N
TOEPLITZ = [
    (1000, 2048, 1),     # single pass
    (3000, 8192, 2),     # power of two, folded
    (30000, 65536, 16),  # power of two, separate strided pass
    (10000, 20480, 5),   # mixed, folded
    (22000, 49152, 12),  # mixed, separate pass, one thread per column
    (45000, 98304, 24),  # mixed, separate pass, thread pairs
]


def toeplitz_case(prec, n, ncols, seed, select=None):
    rng = np.random.default_rng(seed)
    col, row = crandn(rng, n, NP[prec]), crandn(rng, n, NP[prec])
    xt = np.zeros((ncols, n), np.complex128)
    for j in range(ncols):
        k = max(n // 256, 2)
        xt[j, rng.choice(n, k, replace=False)] = rng.standard_normal(k)
    emb = p2(2 * n - 1)
    ap = lambda v: structured.toeplitz_apply_fft64(col, row, v, L=emb)
    ad = lambda v: structured.toeplitz_apply_fft64(col, row, v, True, L=emb)
    rows = None
    if select is not None:
        rows = np.sort(rng.choice(n, select, replace=False)).astype(np.int64)
        ap0, ad0 = ap, ad

        def ap(v):
            return ap0(v)[:, rows]

        def ad(u):
            z = np.zeros((u.shape[0], n), np.complex128)
            z[:, rows] = u
            return ad0(z)
    m = n if rows is None else rows.size
    b = (ap(xt) + 1e-3 * crandn(rng, (ncols, m), np.complex128)).astype(NP[prec])
    # step constant: max |DFT of the embedded generator|^2 bounds ||T||^2 (and ||S T||^2)
    g = np.zeros(emb, np.complex128)
    g[:n] = col
    g[emb - n + 1:] = row[1:][::-1]
    L = float(np.max(np.abs(np.fft.fft(g))) ** 2)
    return col, row, rows, b, ap, ad, L


@pytest.mark.parametrize("prec", ["c64", "c128"])
@pytest.mark.parametrize("n,L_expect,n2", TOEPLITZ)
@pytest.mark.parametrize("select", [False, True])
def test_toeplitz_forms(gpu, prec, n, L_expect, n2, select):
    import torch

    ncols, iters = 3, 30
    col, row, rows, b, ap, ad, L = toeplitz_case(prec, n, ncols, seed=n + select,
                                                  select=(n // 4 if select else None))
    T = gpu.Toeplitz(to_dev(col), to_dev(row))
    assert T.transform_length == L_expect
    A = T if rows is None else gpu.Product(gpu.SelectRows(n, to_dev(rows.astype(np.int32)), tdt(prec)), T)
    lam = 0.05 * float(np.max(np.abs(ad(b.astype(np.complex128)))))
    x, st = gpu.fista(A, to_dev(b), iters=iters, lam=lam, L=L)
    assert all(s["iters"] == iters and s["status"] == 0 for s in st)
    x_ref, _ = fista.fista_op(ap, ad, n, b, lam, L, iters)
    err = rel_err(to_host(x), x_ref)
    assert err <= TOL[prec], f"N={n} L={L_expect} select={select} {prec}: {err:.3e}"


@pytest.mark.parametrize("prec", ["c64", "c128"])
@pytest.mark.parametrize("n", [16, 1024, 65536])
def test_circulant_ista_and_fista(gpu, prec, n):
    rng = np.random.default_rng(n)
    c = crandn(rng, n, NP[prec])
    rows = np.sort(rng.choice(n, n // 8, replace=False)).astype(np.int32)
    ap, ad = structured.select_circulant_fft64(c.astype(np.complex128), rows)
    xt = np.zeros((2, n), np.complex128)
    for j in range(2):
        xt[j, rng.choice(n, max(n // 64, 1), replace=False)] = rng.standard_normal(max(n // 64, 1))
    b = (ap(xt) + 1e-3 * crandn(rng, (2, rows.size), np.complex128)).astype(NP[prec])
    L = float(np.max(np.abs(np.fft.fft(c.astype(np.complex128)))) ** 2)
    lam = 0.05 * float(np.max(np.abs(ad(b.astype(np.complex128)))))
    A = gpu.Product(gpu.SelectRows(n, to_dev(rows), tdt(prec)), gpu.Circulant(to_dev(c)))
    for momentum in (True, False):
        x, _ = gpu.fista(A, to_dev(b), iters=25, momentum=momentum, lam=lam, L=L)
        x_ref, _ = fista.fista_op(ap, ad, n, b, lam, L, 25, momentum=momentum)
        assert rel_err(to_host(x), x_ref) <= TOL[prec], (n, prec, momentum)


@pytest.mark.parametrize("prec", ["c64", "c128"])
@pytest.mark.parametrize("n,iters", [(65536, 30), (262144, 20), (1048576, 8)])
def test_select_circulant_row_lengths(gpu, prec, n, iters):
    """A = S C of power-of-two length L >= 65536: one or two columns run the
    split with 1024-point rows (n2 = L / 1024 = 64 .. 1024), three columns
    keep 4096-point rows. Both against the oracle, and each narrow column
    against the same column of the three-column solve."""
    rng = np.random.default_rng(n + 5)
    c = crandn(rng, n, NP[prec])
    rows = np.sort(rng.choice(n, n // 16, replace=False)).astype(np.int32)
    ap, ad = structured.select_circulant_fft64(c.astype(np.complex128), rows)
    xt = np.zeros((3, n), np.complex128)
    for j in range(3):
        xt[j, rng.choice(n, 64, replace=False)] = rng.standard_normal(64)
    b = (ap(xt) + 1e-3 * crandn(rng, (3, rows.size), np.complex128)).astype(NP[prec])
    L = float(np.max(np.abs(np.fft.fft(c.astype(np.complex128)))) ** 2)
    lam = 0.05 * float(np.max(np.abs(ad(b.astype(np.complex128)))))
    A = gpu.Product(gpu.SelectRows(n, to_dev(rows), tdt(prec)), gpu.Circulant(to_dev(c)))
    x_ref, _ = fista.fista_op(ap, ad, n, b, lam, L, iters)
    x3, _ = gpu.fista(A, to_dev(b), iters=iters, lam=lam, L=L)
    x3 = to_host(x3)
    assert rel_err(x3, x_ref) <= TOL[prec], (n, prec, "three columns")
    for sl in (slice(0, 1), slice(1, 3)):
        x1, st = gpu.fista(A, to_dev(np.ascontiguousarray(b[sl])), iters=iters, lam=lam, L=L)
        assert all(s_["iters"] == iters and s_["status"] == 0 for s_ in st)
        x1 = to_host(x1)
        assert rel_err(x1, x_ref[sl]) <= TOL[prec], (n, prec, sl)
        assert rel_err(x1, x3[sl]) <= TOL[prec], (n, prec, sl)


def test_stop_counts_and_warm_start_fused(gpu):
    """Per-column stopping and a warm start on a four-step form (complex128:
    the stop decision is taken on values within 1e-12 of the oracle's)."""
    n = 3000
    col, row, rows, b, ap, ad, L = toeplitz_case("c128", n, 3, seed=77, select=1200)
    A = gpu.Product(gpu.SelectRows(n, to_dev(rows.astype(np.int32)), tdt("c128")),
                    gpu.Toeplitz(to_dev(col), to_dev(row)))
    lam = 0.05 * float(np.max(np.abs(ad(b))))
    x, st = gpu.fista(A, to_dev(b), iters=500, lam=lam, L=L, stop_tol=1e-5)
    x_ref, done = fista.fista_op(ap, ad, n, b, lam, L, 500, stop_tol=1e-5)
    counts = np.array([s["iters"] for s in st])
    assert np.all(np.abs(counts - done) <= 1) and np.all(done < 500), (counts, done)
    for j in range(3):
        xj, _ = fista.fista_op(ap, ad, n, b[j:j + 1], lam, L, int(counts[j]))
        assert rel_err(to_host(x)[j:j + 1], xj) <= TOL["c128"]
    x0 = crandn(np.random.default_rng(3), (1, n), np.complex128)
    x, _ = gpu.fista(A, to_dev(b[:1]), iters=12, lam=lam, L=L, x0=to_dev(x0))
    x_ref, _ = fista.fista_op(ap, ad, n, b[:1], lam, L, 12, x0=x0)
    assert rel_err(to_host(x), x_ref) <= TOL["c128"]


def test_stop_counts_short_runs_and_warm_start_chained(gpu):
    """The chained form (a separate power-of-two strided pass, n2 = 16: each
    iteration's stop check runs inside the next iteration's first launch and
    a stop kernel follows the last one): per-column stopping against the
    oracle's counts, runs of 1 and 2 iterations, and a warm start
    (complex128: the stop decision is taken on values within 1e-12 of the
    oracle's)."""
    n = 30000
    col, row, rows, b, ap, ad, L = toeplitz_case("c128", n, 2, seed=78, select=12000)
    T = gpu.Toeplitz(to_dev(col), to_dev(row))
    assert T.transform_length == 65536
    A = gpu.Product(gpu.SelectRows(n, to_dev(rows.astype(np.int32)), tdt("c128")), T)
    lam = 0.05 * float(np.max(np.abs(ad(b))))
    x, st = gpu.fista(A, to_dev(b), iters=400, lam=lam, L=L, stop_tol=1e-4)
    _, done = fista.fista_op(ap, ad, n, b, lam, L, 400, stop_tol=1e-4)
    counts = np.array([s["iters"] for s in st])
    assert np.all(np.abs(counts - done) <= 1) and np.all(done < 400), (counts, done)
    for j in range(2):
        xj, _ = fista.fista_op(ap, ad, n, b[j:j + 1], lam, L, int(counts[j]))
        assert rel_err(to_host(x)[j:j + 1], xj) <= TOL["c128"]
    for iters in (1, 2):
        x, st = gpu.fista(A, to_dev(b), iters=iters, lam=lam, L=L)
        assert all(s["iters"] == iters for s in st)
        x_ref, _ = fista.fista_op(ap, ad, n, b, lam, L, iters)
        assert rel_err(to_host(x), x_ref) <= TOL["c128"], iters
    x0 = crandn(np.random.default_rng(4), (1, n), np.complex128)
    x, _ = gpu.fista(A, to_dev(b[:1]), iters=12, lam=lam, L=L, x0=to_dev(x0))
    x_ref, _ = fista.fista_op(ap, ad, n, b[:1], lam, L, 12, x0=x0)
    assert rel_err(to_host(x), x_ref) <= TOL["c128"]


def test_general_loop_form(gpu):
    """Diag times Circulant has no fused form: the general loop solves it."""
    rng = np.random.default_rng(5)
    n = 512
    c, d = crandn(rng, n), crandn(rng, n)
    A = gpu.Product(gpu.Diag(to_dev(d)), gpu.Circulant(to_dev(c)))
    ap = lambda v: d[None, :].astype(np.complex128) * structured.circulant_apply_fft64(c, v)
    ad = lambda u: structured.circulant_apply_fft64(c, np.conj(d)[None, :].astype(np.complex128) * u, True)
    b = crandn(rng, (2, n))
    L = float(np.max(np.abs(d.astype(np.complex128))) ** 2 * np.max(np.abs(np.fft.fft(c.astype(np.complex128)))) ** 2)
    lam = 0.05 * float(np.max(np.abs(ad(b.astype(np.complex128)))))
    x, _ = gpu.fista(A, to_dev(b), iters=20, lam=lam, L=L)
    x_ref, _ = fista.fista_op(ap, ad, n, b, lam, L, 20)
    assert rel_err(to_host(x), x_ref) <= TOL["c64"]
