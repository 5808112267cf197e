"""Pins for the gradient oracle (circulant generator gradient, soft-threshold
derivative, CPU float64 autograd through dense unrolled FISTA).

Checks: the correlation formula against torch autograd of the dense product
built by indexing the generator, the adjoint identity with the dense circulant
of the ``dense`` tier, finite differences (torch.autograd.gradcheck) through
the soft threshold and through the whole unrolled solver, the closed-form
soft-threshold derivative against autograd, and the dense unrolled forward
against the NumPy solver oracle.
"""

import numpy as np
import pytest
import torch

from oracle import dense, fista, grad

RNG = np.random.default_rng(2024)


def crand(*shape):
    return (RNG.standard_normal(shape) + 1j * RNG.standard_normal(shape)) / np.sqrt(2)


def test_circulant_t_matches_dense_definition():
    c = crand(9)
    assert np.array_equal(grad.circulant_t(torch.tensor(c)).numpy(), dense.circulant(c))
    rows = np.array([0, 3, 4, 8])
    assert np.array_equal(grad.selected_circulant_t(torch.tensor(c), rows).numpy(), dense.circulant(c)[rows])


@pytest.mark.parametrize("adjoint", [False, True])
def test_generator_grad_equals_autograd(adjoint):
    n, ncols = 8, 3
    c, x, g = crand(n), crand(ncols, n), crand(ncols, n)
    ct = torch.tensor(c, requires_grad=True)
    C = grad.circulant_t(ct)
    y = torch.tensor(x) @ (C.conj() if adjoint else C.T)  # rows: C x_j or C^H x_j
    (gc,) = torch.autograd.grad(y, ct, grad_outputs=torch.tensor(g))
    assert np.allclose(grad.generator_grad(adjoint, x, g), gc.numpy(), rtol=0, atol=1e-13)


def test_generator_grad_adjoint_identity():
    # y = C(c) x is linear in c with matrix C(x): <g, C(x) c'> = <grad_c, c'>
    n, ncols = 16, 4
    x, g, cp = crand(ncols, n), crand(ncols, n), crand(n)
    gc = grad.generator_grad(False, x, g)
    lhs = sum(np.vdot(g[j], dense.circulant(x[j]) @ cp) for j in range(ncols))
    assert abs(lhs - np.vdot(gc, cp)) <= 1e-12 * np.linalg.norm(gc) * np.linalg.norm(cp)
    # w = C(c)^H u is linear in conj(c): <g, w(c')> = <c', grad_c> (conjugated pairing)
    u = crand(ncols, n)
    ga = grad.generator_grad(True, u, g)
    lhs = sum(np.vdot(g[j], dense.circulant(cp).conj().T @ u[j]) for j in range(ncols))
    assert abs(lhs - np.vdot(cp, ga)) <= 1e-12 * np.linalg.norm(ga) * np.linalg.norm(cp)


def test_correlation_special_cases():
    n = 8
    e0 = np.zeros(n, complex)
    e0[0] = 1
    b = crand(n)
    # a = delta: r[k] = conj(b[-k mod n])
    r = grad.correlation(e0, b)
    assert np.allclose(r, np.conj(b[(-np.arange(n)) % n]), atol=1e-15)
    # autocorrelation at lag 0 is the squared norm
    assert abs(grad.correlation(b, b)[0] - np.vdot(b, b)) < 1e-14


def test_soft_vjp_closed_form_equals_autograd():
    z = crand(2, 50) * 2
    s = np.array([[0.7], [1.1]])
    gout = crand(2, 50)
    zt = torch.tensor(z, requires_grad=True)
    out = grad.soft_t(zt, torch.tensor(s))
    (gz,) = torch.autograd.grad(out, zt, grad_outputs=torch.tensor(gout))
    assert np.allclose(grad.soft_vjp(z, s, gout), gz.numpy(), rtol=0, atol=1e-14)
    # forward of soft_t is the oracle's soft threshold
    assert np.allclose(out.detach().numpy(), fista.soft(z, s), rtol=0, atol=1e-15)


def test_soft_vjp_degenerate_points():
    s = 0.5
    z = np.array([0.0, 0.5, 0.3 + 0.4j, 0.2])  # zero, on the threshold (|z| = s twice), inside
    assert np.all(grad.soft_vjp(z, s, np.ones(4)) == 0)


def test_soft_gradcheck():
    z = torch.tensor(crand(12) * 3)
    s = 0.4
    keep = np.abs(z.numpy())
    z = z[torch.tensor(np.abs(keep - s) > 0.05)].clone().requires_grad_(True)
    assert torch.autograd.gradcheck(lambda t: grad.soft_t(t, s), (z,), eps=1e-7, atol=1e-6)


def test_unrolled_forward_equals_solver_oracle():
    n, rows = 32, np.sort(RNG.choice(32, 12, replace=False))
    c, b = crand(n), crand(3, 12)
    a = dense.product(dense.select_rows(n, rows), dense.circulant(c))
    L = fista.spectral_norm_sq(a)
    lam = fista.lambda_rule(a, b, 0.1)
    x_ref, _ = fista.fista(a, b, lam, L, 15)
    x = grad.unrolled_fista_t(grad.selected_circulant_t(torch.tensor(c), rows), torch.tensor(b), lam, L, 15)
    assert np.allclose(x.numpy(), x_ref, rtol=0, atol=1e-12)


def test_unrolled_gradcheck():
    """Finite differences through 6 unrolled FISTA steps in c and b."""
    n = 16
    rows = np.array([0, 2, 3, 7, 9, 12, 13, 15])
    rng = np.random.default_rng(5)
    c = (rng.standard_normal(n) + 1j * rng.standard_normal(n)) / np.sqrt(2)
    b = (rng.standard_normal((2, 8)) + 1j * rng.standard_normal((2, 8))) / np.sqrt(2)
    a = dense.product(dense.select_rows(n, rows), dense.circulant(c))
    L = 1.5 * fista.spectral_norm_sq(a)
    lam = fista.lambda_rule(a, b, 0.2)
    _, _, _, margin = grad.unrolled_fista_grads(c, b, rows, lam, L, 6, np.ones((2, n)))
    assert margin > 1e-3  # no |z| near the threshold: the map is smooth there

    def f(ct, bt):
        return grad.unrolled_fista_t(grad.selected_circulant_t(ct, rows), bt, lam, L, 6)

    ct = torch.tensor(c, requires_grad=True)
    bt = torch.tensor(b, requires_grad=True)
    assert torch.autograd.gradcheck(f, (ct, bt), eps=1e-7, atol=1e-6)
