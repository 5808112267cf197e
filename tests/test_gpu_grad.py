"""GPU parity of the differentiation path against the gradient oracle.

Generator gradient (fm_circulant_grad_generator) against the correlation
written from its definition; the FISTA step and its vector-Jacobian product
against the oracle's step and closed-form soft-threshold derivative; the
structural norm bound against closed forms; the torch.autograd.Functions
(operator application, circulant application, checkpointed unrolled FISTA)
against CPU float64 autograd through dense matrices. Tolerances: relative L2
per column <= 2e-5 (complex64) and <= 1e-12 (complex128), for single
operations and for gradients through 20 unrolled steps alike.
"""

import numpy as np
import pytest

from oracle import dense, fista, grad, structured
from tests.gpu_util import TOL, crandn, rel_err, to_dev, to_host

pytestmark = pytest.mark.gpu

NP = {"c64": np.complex64, "c128": np.complex128}


def tdt(prec):
    import torch

    return {"c64": torch.complex64, "c128": torch.complex128}[prec]


# ---------------------------------------------------------------- generator gradient
@pytest.mark.parametrize("prec", ["c64", "c128"])
@pytest.mark.parametrize("n,ncols", [(8, 1), (1024, 5), (8192, 3)])
@pytest.mark.parametrize("adjoint", [False, True])
def test_generator_grad(gpu, prec, n, ncols, adjoint):
    rng = np.random.default_rng(n + ncols)
    inp, g = crandn(rng, (ncols, n), NP[prec]), crandn(rng, (ncols, n), NP[prec])
    ref = grad.generator_grad(adjoint, inp, g)
    out = gpu.autograd.grad_generator(to_dev(inp), to_dev(g), adjoint)
    assert rel_err(to_host(out), ref) <= TOL[prec]
    # accumulate adds to what is there
    base = crandn(rng, n, NP[prec])
    out = to_dev(base)
    gpu.autograd.grad_generator(to_dev(inp), to_dev(g), adjoint, out=out, accumulate=True)
    assert rel_err(to_host(out), ref + base) <= TOL[prec]


@pytest.mark.parametrize("prec,n,ncols", [("c64", 65536, 7), ("c128", 65536, 3), ("c64", 1 << 20, 20)])
def test_generator_grad_four_step_sampled_lags(gpu, prec, n, ncols):
    """Four-step lengths (spectra kept in the split's order) and, at 2^20
    with 20 columns, more columns than one internal chunk: lags sampled from
    the correlation's definition r[k] = sum_j sum_i a_j[i] conj(b_j[i - k])."""
    rng = np.random.default_rng(n + ncols + 1)
    inp, g = crandn(rng, (ncols, n), NP[prec]), crandn(rng, (ncols, n), NP[prec])
    lags = np.concatenate([[0, 1, n - 1], rng.choice(np.arange(2, n - 1), 5, replace=False)])
    for adjoint in (False, True):
        a, b = (inp, g) if adjoint else (g, inp)
        a64, b64 = a.astype(np.complex128), b.astype(np.complex128)
        ref = np.array([np.sum(a64 * np.conj(np.roll(b64, k, axis=1))) for k in lags])
        out = to_host(gpu.autograd.grad_generator(to_dev(inp), to_dev(g), adjoint))
        assert rel_err(out[lags], ref) <= TOL[prec], adjoint


def test_generator_grad_zero_columns_and_errors(gpu):
    import torch

    from paper_1710_09578_amd import capi

    out = to_dev(np.ones(16, np.complex64))
    capi.fm_circulant_grad_generator(16, 0, capi.FM_FWD, None, 16, None, 16, out, 0, capi.FM_C64, 0)
    assert np.all(to_host(out) == 0)
    x = torch.zeros((2, 12), dtype=torch.complex64, device="cuda")
    with pytest.raises(capi.FmError) as e:
        gpu.autograd.grad_generator(x, x, False)
    assert e.value.code == "FM_E_UNSUPPORTED"
    x = torch.zeros((2, 16), dtype=torch.complex64, device="cuda")
    with pytest.raises(capi.FmError) as e:  # gradient inside an input block
        capi.fm_circulant_grad_generator(16, 2, capi.FM_FWD, x, 16, x, 16, x[1], 0, capi.FM_C64, 0)
    assert e.value.code == "FM_E_ALIAS"


# ---------------------------------------------------------------- FISTA step and its VJP
@pytest.mark.parametrize("prec", ["c64", "c128"])
def test_fista_step_and_vjp(gpu, prec):
    import torch

    from paper_1710_09578_amd import capi

    rng = np.random.default_rng(3)
    n, ncols, L, k = 1000, 3, 2.5, 6
    beta = fista.momentum_sequence(k + 1)[1][k]  # the oracle's weight of iteration k
    assert abs(capi.fm_fista_momentum(k, 1) - beta) <= 1e-15 and capi.fm_fista_momentum(k, 0) == 0.0
    y, g, xo = (crandn(rng, (ncols, n), NP[prec]) for _ in range(3))
    lam = np.array([0.5, 1.0, 2.0])
    dy, dg, dxo = to_dev(y), to_dev(g), to_dev(xo)
    xn, yn, z = (torch.empty_like(dy) for _ in range(3))
    dl = to_dev(lam)
    dt = capi.FM_C64 if prec == "c64" else capi.FM_C128
    capi.fm_fista_step(n, ncols, dy, dg, dxo, xn, yn, z, n, dl, L, k, 1, dt, 0)
    y64, g64, xo64 = (a.astype(np.complex128) for a in (y, g, xo))
    z_ref = y64 - g64 / L
    x_ref = fista.soft(z_ref, lam[:, None] / L)
    y_ref = x_ref + beta * (x_ref - xo64)
    for got, ref in ((z, z_ref), (xn, x_ref), (yn, y_ref)):
        assert rel_err(to_host(got), ref) <= TOL[prec]
    # VJP: upstream gradients of x_new and y_new
    gx, gy = crandn(rng, (ncols, n), NP[prec]), crandn(rng, (ncols, n), NP[prec])
    dgx, dgy = to_dev(gx), to_dev(gy)
    gz, gg, gxo = (torch.empty_like(dy) for _ in range(3))
    capi.fm_fista_step_vjp(n, ncols, z, dgx, dgy, gz, gg, gxo, n, dl, L, k, 1, dt, 0)
    zh = to_host(z).astype(np.complex128)  # the same z on both sides
    xt = gx.astype(np.complex128) + (1 + beta) * gy.astype(np.complex128)
    gz_ref = grad.soft_vjp(zh, lam[:, None] / L, xt)
    assert rel_err(to_host(gz), gz_ref) <= TOL[prec]
    assert rel_err(to_host(gg), -gz_ref / L) <= TOL[prec]
    assert rel_err(to_host(gxo), -beta * gy.astype(np.complex128)) <= TOL[prec]
    # in place: gz into gx_new, gx_old into gy_new
    capi.fm_fista_step_vjp(n, ncols, z, dgx, dgy, dgx, None, dgy, n, dl, L, k, 1, dt, 0)
    assert rel_err(to_host(dgx), gz_ref) <= TOL[prec]
    assert rel_err(to_host(dgy), -beta * gy.astype(np.complex128)) <= TOL[prec]


def test_axpby(gpu):
    from paper_1710_09578_amd import capi

    rng = np.random.default_rng(4)
    x, y = crandn(rng, (3, 77), np.complex128), crandn(rng, (3, 77), np.complex128)
    dx, dy = to_dev(x), to_dev(y)
    capi.fm_axpby(77, 3, 2.0, dx, 77, -0.5, dy, 77, dx, 77, capi.FM_C128, 0)
    assert rel_err(to_host(dx), 2 * x - 0.5 * y) <= 1e-15


# ---------------------------------------------------------------- structural norm bound
def test_norm_bound(gpu):
    import torch

    from paper_1710_09578_amd import capi

    rng = np.random.default_rng(6)
    c = crandn(rng, 256)
    col, row = crandn(rng, 300), crandn(rng, 200)
    d = crandn(rng, 50)
    gm = crandn(rng, (6, 4))
    rows = np.sort(rng.choice(256, 64, replace=False)).astype(np.int32)
    C = gpu.Circulant(to_dev(c))
    T = gpu.Toeplitz(to_dev(col), to_dev(row))
    cases = [
        (gpu.Fourier(64), 64.0),
        (gpu.Hadamard(32), 32.0),
        (C, np.max(np.abs(np.fft.fft(c.astype(np.complex128)))) ** 2),
        (gpu.Product(gpu.SelectRows(256, to_dev(rows)), C), np.max(np.abs(np.fft.fft(c.astype(np.complex128)))) ** 2),
        (gpu.Diag(to_dev(d)), np.max(np.abs(d.astype(np.complex128))) ** 2),
        (gpu.Dense(to_dev(gm)), np.sum(np.abs(gm.astype(np.complex128)) ** 2)),
        (gpu.Kron(gpu.Fourier(8), gpu.Hadamard(4)), 32.0),
        (gpu.Sum(gpu.Fourier(16), gpu.Fourier(16)), 64.0),
    ]
    L = 512
    g = np.zeros(L, np.complex128)
    g[:300] = col
    g[L - 199:] = row[1:][::-1]
    cases.append((T, np.max(np.abs(np.fft.fft(g))) ** 2))
    for op, ref in cases:
        v = capi.fm_op_norm_bound(op.handle, 0)
        assert abs(v - ref) <= 1e-12 * ref, (op, v, ref)
    # it bounds the spectral norm from above
    a = dense.toeplitz(col, row)
    assert capi.fm_op_norm_bound(T.handle, 0) >= np.linalg.norm(a, 2) ** 2 * (1 - 1e-12)
    del torch


# ---------------------------------------------------------------- autograd functions
@pytest.mark.parametrize("prec", ["c64", "c128"])
def test_operator_apply_autograd(gpu, prec):
    import torch

    rng = np.random.default_rng(8)
    col, row = crandn(rng, 300, NP[prec]), crandn(rng, 200, NP[prec])
    T = gpu.Toeplitz(to_dev(col), to_dev(row))
    a = dense.toeplitz(col, row)
    x = to_dev(crandn(rng, (4, 200), NP[prec])).requires_grad_(True)
    g = crandn(rng, (4, 300), NP[prec])
    y = gpu.autograd.apply(T, x)
    (gx,) = torch.autograd.grad(y, x, grad_outputs=to_dev(g))
    assert rel_err(to_host(gx), dense.apply(a, g, True)) <= TOL[prec]
    w = gpu.autograd.apply(T, to_dev(g).requires_grad_(True), adjoint=True)
    assert w.shape == (4, 200)


@pytest.mark.parametrize("prec", ["c64", "c128"])
@pytest.mark.parametrize("adjoint", [False, True])
def test_circulant_apply_autograd(gpu, prec, adjoint):
    import torch

    rng = np.random.default_rng(9)
    n = 512
    c, x, g = crandn(rng, n, NP[prec]), crandn(rng, (3, n), NP[prec]), crandn(rng, (3, n), NP[prec])
    ct = to_dev(c).requires_grad_(True)
    xt = to_dev(x).requires_grad_(True)
    y = gpu.autograd.circulant_apply(ct, xt, adjoint)
    gc, gx = torch.autograd.grad(y, (ct, xt), grad_outputs=to_dev(g))
    # oracle: CPU float64 autograd through the dense product
    cc = torch.tensor(c.astype(np.complex128), requires_grad=True)
    xx = torch.tensor(x.astype(np.complex128), requires_grad=True)
    C = grad.circulant_t(cc)
    yy = xx @ (C.conj() if adjoint else C.T)
    rc, rx = torch.autograd.grad(yy, (cc, xx), grad_outputs=torch.tensor(g.astype(np.complex128)))
    assert rel_err(to_host(y), yy.detach().numpy()) <= TOL[prec]
    assert rel_err(to_host(gc), rc.numpy()) <= TOL[prec]
    assert rel_err(to_host(gx), rx.numpy()) <= TOL[prec]


def _unrolled_case(n, m, ncols, k, seed, prec):
    rng = np.random.default_rng(seed)
    c = crandn(rng, n, NP[prec])
    rows = np.sort(rng.choice(n, m, replace=False)).astype(np.int32)
    xt = np.zeros((ncols, n), np.complex128)
    for j in range(ncols):
        xt[j, rng.choice(n, k, replace=False)] = rng.standard_normal(k)
    a_sel = structured.select_circulant_fft64(c.astype(np.complex128), rows)
    b = (a_sel[0](xt) + 1e-3 * crandn(rng, (ncols, m), np.complex128)).astype(NP[prec])
    lam = 0.05 * np.max(np.abs(a_sel[1](b.astype(np.complex128))), axis=1)
    L = float(np.max(np.abs(np.fft.fft(c.astype(np.complex128)))) ** 2)
    gout = crandn(rng, (ncols, n), NP[prec])
    return c, rows, b, lam, L, gout


@pytest.mark.parametrize("prec,n,m,ncols,ckpt", [
    ("c128", 64, 24, 3, 5),
    ("c128", 64, 24, 3, 3),   # ragged last segment (20 = 6*3 + 2)
    ("c128", 64, 24, 2, 1),
    ("c64", 1024, 256, 4, 5),
])
def test_unrolled_fista_gradients(gpu, prec, n, m, ncols, ckpt):
    import torch

    c, rows, b, lam, L, gout = _unrolled_case(n, m, ncols, max(n // 32, 2), n + ncols, prec)
    x_ref, gc_ref, gb_ref, margin = grad.unrolled_fista_grads(c, b, rows, lam, L, 20, gout)
    ct = to_dev(c).requires_grad_(True)
    bt = to_dev(b).requires_grad_(True)
    x = gpu.autograd.unrolled_fista(ct, bt, to_dev(rows), to_dev(lam), L=L, iters=20, checkpoint=ckpt)
    gc, gb = torch.autograd.grad(x, (ct, bt), grad_outputs=to_dev(gout))
    ex, ec, eb = rel_err(to_host(x), x_ref), rel_err(to_host(gc), gc_ref), rel_err(to_host(gb), gb_ref)
    msg = f"unrolled {prec} n={n}: x {ex:.2e} grad_c {ec:.2e} grad_b {eb:.2e} (threshold margin {margin:.1e})"
    print(msg)
    assert ex <= TOL[prec] and ec <= TOL[prec] and eb <= TOL[prec], msg


def test_unrolled_fista_default_step_and_scalar_lambda(gpu):
    import torch

    c, rows, b, lam, L, gout = _unrolled_case(64, 24, 2, 3, 11, "c128")
    lam0 = float(lam[0])
    x_ref, gc_ref, _, _ = grad.unrolled_fista_grads(c, b, rows, np.full(2, lam0), L, 10, gout)
    ct = to_dev(c).requires_grad_(True)
    x = gpu.autograd.unrolled_fista(ct, to_dev(b), to_dev(rows), lam0, iters=10)  # L from the norm bound
    (gc,) = torch.autograd.grad(x, ct, grad_outputs=to_dev(gout))
    assert rel_err(to_host(x), x_ref) <= 1e-12 and rel_err(to_host(gc), gc_ref) <= 1e-12


@pytest.mark.parametrize("prec", ["c64", "c128"])
def test_learn_circulant_full_size_sampled_pairs(gpu, prec):
    """N = 16384, M = 2048, 20 unrolled steps (checkpoints every 5), 8 of the
    256 pairs (each pair's gradient contribution is independent, so the check
    is exact for the pairs taken). Oracle: CPU float64 autograd through the
    dense 2048 x 16384 selected circulant."""
    import torch

    from workloads import learn_circulant

    d = learn_circulant()
    pairs = [0, 37, 64, 101, 150, 199, 230, 255]
    c_true, c, rows = d["c_true"], d["c_init"], d["rows"]
    ap, ad = structured.select_circulant_fft64(c_true.astype(np.complex128), rows)
    xs = d["x"][pairs].astype(np.complex128)
    b = (ap(xs) + d["noise"][pairs]).astype(NP[prec])
    lam = 0.05 * np.max(np.abs(ad(b.astype(np.complex128))), axis=1)
    L = float(np.max(np.abs(np.fft.fft(c.astype(np.complex128)))) ** 2)
    ct = to_dev(c.astype(NP[prec])).requires_grad_(True)
    x = gpu.autograd.unrolled_fista(ct, to_dev(b), to_dev(rows), to_dev(lam), L=L, iters=20, checkpoint=5)
    x_host = to_host(x).astype(np.complex128)
    # loss = mean |x_K - x_p|^2: its gradient in x_K (PyTorch convention) is 2 (x_K - x_p) / size
    gout = (2.0 / xs.size) * (x_host - xs)
    (gc,) = torch.autograd.grad(x, ct, grad_outputs=to_dev(gout.astype(NP[prec])))
    x_ref, gc_ref, _, margin = grad.unrolled_fista_grads(c, b, rows, lam, L, 20, gout)
    ex, ec = rel_err(x_host, x_ref), rel_err(to_host(gc), gc_ref)
    msg = f"learn-circulant 16384 {prec}: x {ex:.2e} grad_c {ec:.2e} (threshold margin {margin:.1e})"
    print(msg)
    assert ex <= TOL[prec] and ec <= TOL[prec], msg
