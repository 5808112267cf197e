"""Orthogonal matching pursuit in FP64 with a dense operator.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The greedy sparse-recovery method the paper runs beside FISTA on the
ultrasound model (section "Application to Ultrasonic Nondestructive
Testing", reconstruction figure; OMP after Tropp and Gilbert). Per column b:

    r = b, S = []
    repeat k times:
        c = A^H r                      (correlations: one backward transform)
        j = argmax_{i not in S} |c_i|  (first index on ties)
        S = S + [j]
        x_S = argmin ||A_S x_S - b||_2 (least squares on the chosen columns)
        r = b - A_S x_S
        stop early when ||r||_2 <= tol ||b||_2
    x = x_S at S, zero elsewhere

Readings (the paper gives no listing): correlations are not normalised by the
column norms (the operators here have columns of equal norm, where the two
agree); a selected index is never selected again; the least-squares solve is
numpy's (a library primitive).

Pins (tests/test_oracle_omp.py): with orthonormal columns OMP keeps the k
largest |A^H b| entries (closed form); the residual is orthogonal to every
chosen column after each step; k = n on a square invertible A gives A^{-1} b;
a noiseless k-sparse vector is recovered exactly by a well-conditioned
Gaussian A.
"""

from __future__ import annotations

import numpy as np

C128 = np.complex128


def omp(a, b, k: int, tol: float = 0.0, history: bool = False):
    """OMP on each column of b (shape (ncols, m)) with the dense A (m, n).

    Returns (x (ncols, n), supports (ncols, k) in selection order with -1 for
    unused slots, atoms per column) and, with history, the residuals after
    every step of every column.
    """
    a = np.asarray(a, dtype=C128)
    b = np.atleast_2d(np.asarray(b, dtype=C128))
    ncols, m = b.shape
    n = a.shape[1]
    x = np.zeros((ncols, n), dtype=C128)
    sup = np.full((ncols, k), -1, dtype=np.int64)
    atoms = np.zeros(ncols, dtype=np.int64)
    hist = []
    for col in range(ncols):
        bc = b[col]
        r = bc.copy()
        chosen: list[int] = []
        xs = np.zeros(0, dtype=C128)
        steps = []
        bnorm = np.linalg.norm(bc)
        for _ in range(k):
            if np.linalg.norm(r) <= tol * bnorm:
                break
            c = a.conj().T @ r
            mag = np.abs(c)
            mag[chosen] = -1.0
            j = int(np.argmax(mag))  # first maximal index
            chosen.append(j)
            xs = np.linalg.lstsq(a[:, chosen], bc, rcond=None)[0]
            r = bc - a[:, chosen] @ xs
            steps.append(r.copy())
        x[col, chosen] = xs
        sup[col, :len(chosen)] = chosen
        atoms[col] = len(chosen)
        hist.append(steps)
    return (x, sup, atoms, hist) if history else (x, sup, atoms)


def least_squares_on(a, b, support):
    """x_S = argmin ||A_S x_S - b|| for a given support (one column of b),
    scattered into a length-n vector."""
    a = np.asarray(a, dtype=C128)
    s = [int(v) for v in support if v >= 0]
    x = np.zeros(a.shape[1], dtype=C128)
    if s:
        x[s] = np.linalg.lstsq(a[:, s], np.asarray(b, dtype=C128), rcond=None)[0]
    return x
