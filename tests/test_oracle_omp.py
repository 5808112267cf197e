"""Pins for the OMP oracle: closed form for orthonormal columns, residual
orthogonality after every step, the exact solve at full support, exact
recovery of a noiseless sparse vector, early stop on the residual tolerance."""

import numpy as np

from oracle import dense, omp

RNG = np.random.default_rng(404)


def crand(*shape):
    return RNG.standard_normal(shape) + 1j * RNG.standard_normal(shape)


def test_orthonormal_columns_keep_largest_coefficients():
    """A = F_n / sqrt(n) is unitary: x_S = A^H b on S and the greedy picks are
    the k largest |A^H b| in decreasing order."""
    n, k = 32, 6
    a = dense.fourier(n) / np.sqrt(n)
    b = crand(2, n)
    x, sup, atoms = omp.omp(a, b, k)
    for col in range(2):
        c = a.conj().T @ b[col]
        order = np.argsort(-np.abs(c), kind="stable")[:k]
        assert list(sup[col]) == list(order)
        ref = np.zeros(n, complex)
        ref[order] = c[order]
        assert np.allclose(x[col], ref, atol=1e-12)
    assert list(atoms) == [k, k]


def test_residual_orthogonal_to_chosen_columns():
    a = crand(40, 70)
    b = crand(1, 40)
    x, sup, atoms, hist = omp.omp(a, b, 10, history=True)
    for step, r in enumerate(hist[0]):
        s = sup[0, :step + 1]
        assert np.max(np.abs(a[:, s].conj().T @ r)) <= 1e-10 * np.linalg.norm(b)
    # residuals decrease monotonically
    norms = [np.linalg.norm(r) for r in hist[0]]
    assert all(u >= v - 1e-12 for u, v in zip(norms, norms[1:]))


def test_full_support_solves_square_system():
    n = 12
    a = crand(n, n) + 4 * np.eye(n)
    b = crand(1, n)
    x, sup, atoms = omp.omp(a, b, n)
    assert atoms[0] == n and sorted(sup[0]) == list(range(n))
    assert np.allclose(x[0], np.linalg.solve(a, b[0]), atol=1e-10)


def test_noiseless_sparse_recovery():
    m, n, k = 96, 256, 5
    a = RNG.standard_normal((m, n)) / np.sqrt(m)
    xt = np.zeros(n, complex)
    supp = RNG.choice(n, k, replace=False)
    xt[supp] = np.sign(RNG.standard_normal(k)) * (1 + RNG.random(k))
    x, sup, atoms = omp.omp(a, (a @ xt)[None, :], k)
    assert sorted(sup[0]) == sorted(supp)
    assert np.allclose(x[0], xt, atol=1e-10)
    assert np.allclose(omp.least_squares_on(a, a @ xt, sup[0]), xt, atol=1e-10)


def test_tolerance_stops_early():
    n = 16
    a = dense.fourier(n) / np.sqrt(n)
    xt = np.zeros(n, complex)
    xt[[2, 9]] = [3.0, -2.0]
    b = (a @ xt)[None, :]
    x, sup, atoms = omp.omp(a, b, 8, tol=1e-9)
    assert atoms[0] == 2 and list(sup[0, 2:]) == [-1] * 6
    assert np.allclose(x[0], xt, atol=1e-12)
