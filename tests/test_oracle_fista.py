"""Pins for the solver oracle (soft thresholding, FISTA / ISTA, power
iteration, regularisation rule).

Checks: hand-derived fixtures, the proximal optimality of soft thresholding on
a brute-force grid, closed-form iterates for operators with A^H A = L I, the
exact lasso solution of tiny real problems by enumeration of supports and
signs, KKT conditions at convergence, the Beck-Teboulle rate bound, ISTA's
monotone objective, and closed-form spectral norms for the power iteration.
"""

import itertools
import math

import numpy as np
import pytest

from oracle import dense, fista
from tests.conftest import golden_rows

RNG = np.random.default_rng(99)


def crand(*shape):
    return RNG.standard_normal(shape) + 1j * RNG.standard_normal(shape)


# ---------------------------------------------------------------- soft threshold
def test_soft_golden():
    for zr, zi, s, orr, oi in (map(float, r) for r in golden_rows("soft.txt")):
        out = fista.soft(np.array([zr + 1j * zi]), s)[0]
        assert abs(out - (orr + 1j * oi)) < 1e-15


def test_soft_is_the_prox_on_a_grid():
    # soft(z, s) minimises 1/2 |u - z|^2 + s |u| over complex u
    g = np.linspace(-3, 3, 601)
    u = g[:, None] + 1j * g[None, :]
    for z, s in [(1.3 - 0.7j, 0.4), (0.2 + 0.1j, 0.5), (-2.0 + 1.5j, 1.1)]:
        f = 0.5 * np.abs(u - z) ** 2 + s * np.abs(u)
        best = u.flat[np.argmin(f)]
        assert abs(best - fista.soft(np.array([z]), s)[0]) <= 0.011


def test_momentum_golden():
    rows = {r[0]: [float(v) for v in r[1:]] for r in golden_rows("momentum.txt")}
    t, beta = fista.momentum_sequence(3)
    assert np.allclose(t, rows["t"], rtol=0, atol=1e-15)
    assert np.allclose(beta, rows["beta"], rtol=0, atol=1e-15)


# ---------------------------------------------------------------- FISTA special cases
def test_zero_iterations_return_start():
    a = crand(5, 7)
    b = crand(2, 5)
    x0 = crand(2, 7)
    x, done = fista.fista(a, b, 0.1, 10.0, 0, x0=x0)
    assert np.array_equal(x, x0) and np.all(done == 0)


def test_large_lambda_gives_zero():
    a = crand(6, 9)
    b = crand(3, 6)
    lam_max = fista.lambda_rule(a, b, 1.0)
    L = fista.spectral_norm_sq(a)
    x, _ = fista.fista(a, b, lam_max, L, 50)
    assert np.count_nonzero(x) == 0


def test_lambda_just_below_max_gives_nonzero():
    """The other side of the threshold: for lam slightly below
    ||A^H b||_inf the first step already keeps the largest correlation (x_1 =
    soft(A^H b / L, lam / L) from x_0 = 0), at the index of the largest
    |A^H b|, and the solve stays nonzero. A rule that overstates the maximum
    (e.g. A^T in place of A^H) fails either this test or the one above."""
    a = crand(6, 9)
    b = crand(3, 6)
    lam_max = fista.lambda_rule(a, b, 1.0)
    L = fista.spectral_norm_sq(a)
    lam = (1.0 - 1e-6) * lam_max
    x1, _ = fista.fista(a, b, lam, L, 1)
    corr = np.abs((a.conj().T @ b.T).T)
    for j in range(3):
        nz = np.flatnonzero(x1[j])
        assert nz.tolist() == [int(np.argmax(corr[j]))]
    x, _ = fista.fista(a, b, lam, L, 50)
    assert np.all(np.count_nonzero(x, axis=1) >= 1)
    # the rule itself against a brute-force maximum over every entry of A^H b
    for j in range(3):
        best = max(abs(sum(np.conj(a[i, k]) * b[j, i] for i in range(6))) for k in range(9))
        assert abs(lam_max[j] - best) <= 1e-12 * best


@pytest.mark.parametrize("kind", ["fourier", "hadamard", "kron"])
@pytest.mark.parametrize("momentum", [True, False])
def test_orthogonal_operator_closed_form(kind, momentum):
    a = {"fourier": dense.fourier(16),
         "hadamard": dense.hadamard(16).astype(complex),
         "kron": dense.kron(dense.hadamard(4), dense.fourier(4))}[kind]
    L = 16.0                                      # A^H A = 16 I for all three
    assert np.allclose(a.conj().T @ a, L * np.eye(16))
    b = crand(2, 16)
    lam = np.array([0.5, 3.0])
    expect = fista.soft((a.conj().T @ b.T).T / L, (lam / L)[:, None])
    for k in (1, 2, 7):
        x, _ = fista.fista(a, b, lam, L, k, momentum=momentum)
        assert np.allclose(x, expect, atol=1e-12)


def exact_real_lasso(a, b, lam):
    """Minimiser of 1/2||Ax-b||^2 + lam||x||_1 over real x, by enumerating
    every support and sign pattern (tiny n only)."""
    n = a.shape[1]
    best, best_x = np.inf, None
    for pattern in itertools.product((-1, 0, 1), repeat=n):
        s = np.array(pattern, float)
        supp = np.nonzero(s)[0]
        x = np.zeros(n)
        if supp.size:
            As = a[:, supp]
            xs = np.linalg.solve(As.T @ As, As.T @ b - lam * s[supp])
            if np.any(np.sign(xs) != s[supp]):
                continue
            x[supp] = xs
        grad = a.T @ (b - a @ x)
        off = np.setdiff1d(np.arange(n), supp)
        if np.any(np.abs(grad[off]) > lam + 1e-12):
            continue
        f = 0.5 * np.sum((a @ x - b) ** 2) + lam * np.sum(np.abs(x))
        if f < best:
            best, best_x = f, x
    return best_x, best


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_fista_converges_to_exact_lasso(seed):
    r = np.random.default_rng(seed)
    m, n = 10, 6
    a = r.standard_normal((m, n))
    b = r.standard_normal(m)
    lam = 0.3 * np.max(np.abs(a.T @ b))
    x_star, f_star = exact_real_lasso(a, b, lam)
    L = fista.spectral_norm_sq(a)
    for momentum, iters in ((True, 3000), (False, 20000)):
        x, _ = fista.fista(a.astype(complex), b[None, :].astype(complex), lam, L, iters,
                           momentum=momentum)
        assert np.allclose(x[0].real, x_star, atol=1e-8)
        assert np.allclose(x[0].imag, 0)


def test_kkt_at_convergence_complex():
    a = crand(12, 20)
    b = crand(1, 12)
    lam = 0.2 * fista.lambda_rule(a, b, 1.0)
    L = fista.spectral_norm_sq(a)
    x, _ = fista.fista(a, b, lam, L, 20000)
    x = x[0]
    g = a.conj().T @ (b[0] - a @ x)
    on = np.abs(x) > 1e-10
    assert on.any() and (~on).any()
    assert np.allclose(g[on], lam[0] * x[on] / np.abs(x[on]), atol=1e-7)
    assert np.all(np.abs(g[~on]) <= lam[0] * (1 + 1e-7))


def test_rate_bound_and_ista_monotone():
    a = crand(15, 25)
    b = crand(1, 15)
    lam = 0.1 * fista.lambda_rule(a, b, 1.0)
    L = fista.spectral_norm_sq(a)
    x_star, _ = fista.fista(a, b, lam, L, 30000)
    f_star = fista.objective(a, b, x_star, lam)[0]
    _, _, hist = fista.fista(a, b, lam, L, 200, history=True)
    for k, xk in enumerate(hist, start=1):
        gap = fista.objective(a, b, xk, lam)[0] - f_star
        assert gap <= 2 * L * np.sum(np.abs(x_star) ** 2) / (k + 1) ** 2 + 1e-9
    _, _, hist = fista.fista(a, b, lam, L, 200, momentum=False, history=True)
    fs = [fista.objective(a, b, xk, lam)[0] for xk in hist]
    assert all(fs[i + 1] <= fs[i] + 1e-12 for i in range(len(fs) - 1))


def test_stop_rule_freezes_columns():
    a = crand(8, 8) + 4 * np.eye(8)
    b = crand(3, 8)
    lam = 0.05 * fista.lambda_rule(a, b, 1.0)
    L = fista.spectral_norm_sq(a)
    x_full, _ = fista.fista(a, b, lam, L, 3000)
    x, done = fista.fista(a, b, lam, L, 3000, stop_tol=1e-5)
    assert np.all(done < 3000) and np.all(done > 1)
    # each frozen column equals the plain run stopped at its own count
    for j in range(3):
        xj, _ = fista.fista(a, b[j:j + 1], lam[j], L, int(done[j]))
        assert np.allclose(x[j], xj[0], rtol=0, atol=1e-12)
    assert np.allclose(x, x_full, atol=1e-3 * np.abs(x_full).max())


# ---------------------------------------------------------------- power iteration
@pytest.mark.parametrize("kind", ["circulant", "fourier", "hadamard", "kron", "diag", "random"])
def test_power_iteration_closed_forms(kind):
    n = 32
    if kind == "circulant":
        c = crand(n)
        a, expect = dense.circulant(c), np.max(np.abs(np.fft.fft(c))) ** 2
    elif kind == "fourier":
        a, expect = dense.fourier(n), float(n)
    elif kind == "hadamard":
        a, expect = dense.hadamard(n).astype(complex), float(n)
    elif kind == "kron":
        d = crand(4)
        a = dense.kron(dense.fourier(8), dense.diag(d))
        expect = 8 * np.max(np.abs(d)) ** 2
    elif kind == "diag":
        d = crand(n)
        a, expect = dense.diag(d), np.max(np.abs(d)) ** 2
    else:
        a = crand(20, 30)
        expect = np.linalg.svd(a, compute_uv=False)[0] ** 2
    v0 = crand(a.shape[1])
    L, its = fista.power_iteration(a, v0, max_iters=5000, tol=1e-15)
    assert L <= expect * (1 + 1e-12)
    tol = 1e-12 if kind in ("fourier", "hadamard") else 1e-9
    assert abs(L - expect) <= tol * expect


def test_splitmix64_reference_values():
    expect = [int(r[0], 16) for r in golden_rows("splitmix64.txt")]
    assert fista.splitmix64_outputs(0, 3) == expect
    v = fista.splitmix64_start(3, 0)
    assert v.shape == (3,) and np.all(np.abs(v.real) <= 0.5) and np.all(np.abs(v.imag) <= 0.5)
    assert v[0].real == (expect[0] >> 11) / 2**53 - 0.5


def test_fista_op_matches_dense_form():
    from oracle import structured

    rng = np.random.default_rng(3)
    c = crand(64)
    rows = np.sort(rng.choice(64, 20, replace=False))
    a = dense.product(dense.select_rows(64, rows), dense.circulant(c))
    b = crand(2, 20)
    L = fista.spectral_norm_sq(a)
    lam = fista.lambda_rule(a, b, 0.1)
    ap, ad = structured.select_circulant_fft64(c, rows)
    assert np.allclose(fista.lambda_rule_op(ad, b, 0.1), lam)
    x1, _ = fista.fista(a, b, lam, L, 30)
    x2, _ = fista.fista_op(ap, ad, 64, b, lam, L, 30)
    assert np.allclose(x1, x2, atol=1e-12)
    L2, _ = fista.power_iteration_op(lambda v: ap(v[None])[0], lambda u: ad(u[None])[0],
                                     crand(64), 5000, 1e-15)
    assert abs(L2 - L) <= 1e-9 * L


@pytest.mark.parametrize("embed", [None, 64])
def test_toeplitz_fista_fft64_matches_dense_form(embed):
    """The FFT64 Toeplitz solve (zero-padded cyclic products, any cyclic
    length >= M + N - 1) equals FISTA with the dense Toeplitz matrix, with and
    without per-column stopping."""
    from oracle import structured

    col, row = crand(20), crand(20)
    a = dense.toeplitz(col, row)
    b = crand(3, 20)
    L = fista.spectral_norm_sq(a)
    lam = fista.lambda_rule(a, b, 0.05)
    for tol in (0.0, 1e-5):
        x1, d1 = fista.fista(a, b, lam, L, 60, stop_tol=tol)
        x2, d2 = structured.toeplitz_fista_fft64(col, row, b, lam, L, 60, stop_tol=tol, embed=embed)
        assert np.allclose(x1, x2, atol=1e-12) and np.array_equal(d1, d2)
