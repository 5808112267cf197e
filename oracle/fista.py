"""FISTA / ISTA oracle on dense FP64 operators.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Problem (eq. (8), section "Application to Ultrasonic Nondestructive Testing"),
read with the conventional factor one half: for each column b of a block,

    minimise_x  1/2 ||A x - b||_2^2 + lam ||x||_1

(equivalently tau = 2 lam in eq. (8)); |.| of a complex entry is its modulus.
The paper iterates a soft-thresholded gradient step (ISTA) and uses the
accelerated variant it cites (FISTA, Beck and Teboulle) for its results; both
are implemented here as constant-step proximal-gradient iterations with step
1/L, L >= ||A||_2^2:

    g      = A^H (A y_k - b)
    x_k+1  = soft(y_k - g / L, lam / L)
    t_k+1  = (1 + sqrt(1 + 4 t_k^2)) / 2                 (t_1 = 1)
    y_k+1  = x_k+1 + ((t_k - 1) / t_k+1) (x_k+1 - x_k)   (ISTA: y_k+1 = x_k+1)

starting from x_0 = y_1 = x0 (default zero).
"""

from __future__ import annotations

import math

import numpy as np

C128 = np.complex128


def soft(z, s):
    """Complex soft thresholding tau_s at level s >= 0: shrinks the modulus,
    keeps the phase; entries with |z| <= s become exactly 0 (no division at 0).
    This is the proximal map of s * sum_i |z_i|."""
    z = np.asarray(z, dtype=C128)
    s = np.asarray(s, dtype=np.float64)
    mag = np.abs(z)
    keep = mag > s
    safe = np.where(keep, mag, 1.0)
    return np.where(keep, z * ((mag - s) / safe), 0.0 + 0.0j)


def momentum_sequence(iters: int):
    """t_1 .. t_{iters+1} and the momentum weights (t_k - 1) / t_{k+1}."""
    t = [1.0]
    for _ in range(iters):
        t.append((1.0 + math.sqrt(1.0 + 4.0 * t[-1] * t[-1])) / 2.0)
    beta = [(t[k] - 1.0) / t[k + 1] for k in range(iters)]
    return t, beta


def lambda_rule(a, b, rel: float) -> np.ndarray:
    """lam_j = rel * ||A^H b_j||_inf per column b_j (the regularisation rule of
    the compressed-sensing workloads; ||A^H b||_inf is the smallest lam for
    which x = 0 solves the problem)."""
    a = np.asarray(a, dtype=C128)
    g = (a.conj().T @ np.asarray(b, dtype=C128).T).T
    return rel * np.max(np.abs(g), axis=1)


def objective(a, b, x, lam) -> np.ndarray:
    """1/2 ||A x_j - b_j||^2 + lam_j ||x_j||_1 per column."""
    a = np.asarray(a, dtype=C128)
    r = (a @ np.asarray(x, dtype=C128).T).T - np.asarray(b, dtype=C128)
    return 0.5 * np.sum(np.abs(r) ** 2, axis=1) + np.asarray(lam) * np.sum(np.abs(x), axis=1)


def fista(a, b, lam, L: float, iters: int, momentum: bool = True, x0=None,
          stop_tol: float = 0.0, history: bool = False):
    """Constant-step FISTA (momentum=True) or ISTA (False) with a dense A.

    a: dense (m, n); b: (ncols, m); lam: scalar or (ncols,); L: step constant.
    See ``fista_op`` for the iteration; this form supplies the dense products
    of eq. (2).
    """
    a = np.asarray(a, dtype=C128)
    ah = a.conj().T
    return fista_op(lambda v: (a @ v.T).T, lambda v: (ah @ v.T).T, a.shape[1], b, lam, L, iters,
                    momentum=momentum, x0=x0, stop_tol=stop_tol, history=history)


def fista_op(apply, adjoint, n: int, b, lam, L: float, iters: int, momentum: bool = True,
             x0=None, stop_tol: float = 0.0, history: bool = False):
    """FISTA / ISTA with the operator given by its forward and backward
    transforms (``apply(v)`` = A v, ``adjoint(v)`` = A^H v on blocks of shape
    (ncols, rows)), column by column.

    With stop_tol > 0 a column is frozen after the first iteration k at which
    ||x_k - x_{k-1}||_2 <= stop_tol * max(||x_k||_2, 1e-30); its iterate count
    is then k. Returns (x, iters_done) and, with history, the list of iterates.
    """
    b = np.asarray(b, dtype=C128)
    ncols = b.shape[0]
    lam = np.broadcast_to(np.asarray(lam, dtype=np.float64), (ncols,))
    x_prev = np.zeros((ncols, n), dtype=C128) if x0 is None else np.asarray(x0, dtype=C128).copy()
    y = x_prev.copy()
    _, beta = momentum_sequence(iters)
    done = np.full(ncols, iters, dtype=np.int64)
    active = np.ones(ncols, dtype=bool)
    hist = []
    for k in range(iters):
        g = adjoint(apply(y) - b)
        z = y - g / L
        x = soft(z, (lam / L)[:, None])
        y_new = x + (beta[k] * (x - x_prev) if momentum else 0.0)
        if stop_tol > 0.0:
            dx = np.linalg.norm(x - x_prev, axis=1)
            nx = np.maximum(np.linalg.norm(x, axis=1), 1e-30)
            stop_now = active & (dx <= stop_tol * nx)
        # frozen columns keep their state
        x = np.where(active[:, None], x, x_prev)
        y = np.where(active[:, None], y_new, y)
        x_prev = x
        if stop_tol > 0.0:
            done[stop_now] = k + 1
            active = active & ~stop_now
        if history:
            hist.append(x.copy())
    if history:
        return x_prev, done, hist
    return x_prev, done


def lambda_rule_op(adjoint, b, rel: float) -> np.ndarray:
    """lam_j = rel * ||A^H b_j||_inf with A^H given as a function."""
    return rel * np.max(np.abs(adjoint(np.asarray(b, dtype=C128))), axis=1)


def splitmix64_outputs(seed: int, count: int):
    """The first ``count`` 64-bit outputs of SplitMix64 seeded with ``seed``."""
    mask = (1 << 64) - 1
    out = []
    for k in range(count):
        z = (seed + (k + 1) * 0x9E3779B97F4A7C15) & mask
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & mask
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & mask
        out.append(z ^ (z >> 31))
    return out


def splitmix64_start(n: int, seed: int) -> np.ndarray:
    """Start vector of the power iteration drawn from SplitMix64 (Steele, Lea
    and Flood, 2014): output k of the generator seeded with ``seed`` is the
    finaliser applied to seed + (k+1) * 0x9E3779B97F4A7C15 (mod 2^64); entry i
    is (u(2i) - 1/2) + j (u(2i+1) - 1/2) with u(k) = (output k >> 11) / 2^53."""
    raw = splitmix64_outputs(seed, 2 * n)
    u = np.array([(z >> 11) / float(1 << 53) for z in raw])
    return (u[0::2] - 0.5) + 1j * (u[1::2] - 0.5)


def power_iteration(a, v0, max_iters: int = 500, tol: float = 1e-13):
    """Estimate L = ||A||_2^2 by power iteration on A^H A in FP64 (dense A).

    v <- v0 / ||v0||; repeat: w = A^H (A v); L_k = <v, w> (the Rayleigh
    quotient, = ||A v||^2); v <- w / ||w||; stop when |L_k - L_{k-1}| <=
    tol * L_k or after max_iters. Returns (L, iterations).
    """
    a = np.asarray(a, dtype=C128)
    ah = a.conj().T
    return power_iteration_op(lambda v: a @ v, lambda v: ah @ v, v0, max_iters, tol)


def power_iteration_op(apply, adjoint, v0, max_iters: int = 500, tol: float = 1e-13):
    """The power iteration of ``power_iteration`` with A given by functions
    on single vectors."""
    v = np.asarray(v0, dtype=C128)
    v = v / np.linalg.norm(v)
    prev = None
    lk = 0.0
    for it in range(1, max_iters + 1):
        av = apply(v)
        lk = float(np.vdot(av, av).real)
        w = adjoint(av)
        nw = np.linalg.norm(w)
        if nw == 0.0:
            return 0.0, it
        v = w / nw
        if prev is not None and abs(lk - prev) <= tol * lk:
            return lk, it
        prev = lk
    return lk, max_iters


def spectral_norm_sq(a) -> float:
    """||A||_2^2 as the square of the largest singular value (LAPACK SVD)."""
    return float(np.linalg.norm(np.asarray(a, dtype=C128), 2) ** 2)
