"""Gradients in FP64 on the CPU: the circulant generator gradient written out
from its definition, and CPU torch float64 autograd through dense unrolled
FISTA.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Conventions: PyTorch's gradient convention for complex tensors (for a real
loss and an upstream gradient G of an output s, the gradient of an input z is
G conj(ds/dz) + conj(G) ds/dz*). Blocks are (ncols, rows) arrays. The solver
is the one of eq. (8) with the readings of ``oracle.fista`` (1/2 ||Ax-b||^2,
complex-modulus soft threshold, constant step 1/L, x0 = 0, t1 = 1); L and
lambda are constants (not differentiated).

Pins (tests/test_oracle_grad.py): the correlation formula equals torch
autograd of the dense product C(c) x (built by indexing c), and satisfies the
adjoint identity <g, C(x) c'> = <grad, c'> with the dense circulant of the
``dense`` tier; the dense unrolled forward equals ``fista.fista``; torch's
gradcheck (finite differences) passes through the unrolled solver and the
soft threshold; the closed-form soft-threshold derivative equals autograd.
"""

from __future__ import annotations

import numpy as np


def correlation(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """r[k] = sum_j sum_i a_j[i] conj(b_j[(i - k) mod n]), straight from the
    definition (O(n^2) per column)."""
    a = np.atleast_2d(np.asarray(a, dtype=np.complex128))
    b = np.atleast_2d(np.asarray(b, dtype=np.complex128))
    n = a.shape[1]
    r = np.empty(n, dtype=np.complex128)
    for k in range(n):
        r[k] = np.sum(a * np.conj(np.roll(b, k, axis=1)))  # roll(b, k)[i] = b[(i - k) mod n]
    return r


def generator_grad(use_adjoint: bool, inp: np.ndarray, g: np.ndarray) -> np.ndarray:
    """Gradient of c for y = C(c) inp (use_adjoint False: correlation of g with
    inp) or w = C(c)^H inp (True: correlation of inp with g)."""
    return correlation(inp, g) if use_adjoint else correlation(g, inp)


def soft_vjp(z: np.ndarray, s, gout: np.ndarray) -> np.ndarray:
    """Closed-form vector-Jacobian product of soft(z, s) = z (|z|-s)/|z|
    (|z| > s, else 0): G (1 - s/(2|z|)) + conj(G) s z^2 / (2 |z|^3) where
    |z| > s, 0 elsewhere (including |z| = s)."""
    z = np.asarray(z, dtype=np.complex128)
    gout = np.asarray(gout, dtype=np.complex128)
    s = np.broadcast_to(np.asarray(s, dtype=np.float64), z.shape)
    m = np.abs(z)
    keep = m > s
    ms = np.where(keep, m, 1.0)
    gz = gout * (1 - s / (2 * ms)) + np.conj(gout) * s * z * z / (2 * ms ** 3)
    return np.where(keep, gz, 0)


# ---------------------------------------------------------------- torch float64 autograd
def _torch():
    import torch

    return torch


def circulant_t(c):
    """Dense C(c)[i, j] = c[(i - j) mod n] as a differentiable torch tensor."""
    torch = _torch()
    n = c.shape[0]
    i = torch.arange(n)
    return c[(i[:, None] - i[None, :]) % n]


def soft_t(z, s):
    """soft(z, s) with torch ops, differentiable, no division at |z| <= s."""
    torch = _torch()
    a = z.abs()
    keep = a > s
    a_safe = torch.where(keep, a, torch.ones_like(a))
    return torch.where(keep, z * (1 - s / a_safe), torch.zeros_like(z))


def unrolled_fista_t(A, b, lam, L, iters, momentum=True, return_z=False):
    """x_K of ``iters`` FISTA steps on the dense torch matrix A (m, n) for the
    block b (ncols, m) with per-column weights lam (ncols,), from x0 = 0.
    With return_z, also returns the list of z_k = y_k - g_k/L."""
    torch = _torch()
    ncols = b.shape[0]
    n = A.shape[1]
    x_prev = torch.zeros((ncols, n), dtype=A.dtype)
    y = x_prev
    t = 1.0
    s = (torch.as_tensor(lam, dtype=torch.float64) / L).reshape(-1, 1)
    zs = []
    for _ in range(iters):
        r = y @ A.T - b
        g = r @ A.conj()
        z = y - g / L
        zs.append(z)
        x = soft_t(z, s)
        t_new = (1.0 + (1.0 + 4.0 * t * t) ** 0.5) / 2.0
        beta = (t - 1.0) / t_new if momentum else 0.0
        y = x + beta * (x - x_prev)
        x_prev = x
        t = t_new
    return (x_prev, zs) if return_z else x_prev


def selected_circulant_t(c, rows):
    """Dense S_rows C(c) (rows None: C(c)): entry (r, j) = c[(rows[r] - j) mod n],
    built for the selected rows only."""
    torch = _torch()
    if rows is None:
        return circulant_t(c)
    n = c.shape[0]
    ri = torch.as_tensor(np.asarray(rows, dtype=np.int64))
    return c[(ri[:, None] - torch.arange(n)[None, :]) % n]


def unrolled_fista_grads(c, b, rows, lam, L, iters, gout, momentum=True):
    """Gradients of sum Re<gout, x_K> with respect to c and b (PyTorch's
    convention), with x_K the unrolled FISTA iterate on S_rows C(c).
    Returns (x_K, grad_c, grad_b, min over steps of | |z| - s | / s)."""
    torch = _torch()
    ct = torch.tensor(np.asarray(c, dtype=np.complex128), requires_grad=True)
    bt = torch.tensor(np.asarray(b, dtype=np.complex128), requires_grad=True)
    A = selected_circulant_t(ct, rows)
    x, zs = unrolled_fista_t(A, bt, lam, L, iters, momentum, return_z=True)
    g = torch.tensor(np.asarray(gout, dtype=np.complex128))
    loss = torch.sum((torch.conj(g) * x).real)
    gc, gb = torch.autograd.grad(loss, (ct, bt))
    s = np.asarray(lam, dtype=np.float64).reshape(-1, 1) / L
    margin = min(float(np.min(np.abs(np.abs(z.detach().numpy()) - s) / s)) for z in zs)
    return x.detach().numpy(), gc.numpy(), gb.numpy(), margin
